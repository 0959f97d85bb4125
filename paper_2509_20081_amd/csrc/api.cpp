// C ABI of the scan-integration library: validation, grids, workspaces,
// statistics delivery, batching with captured HIP graphs, readout.
#include <time.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "runtime.h"

using namespace dbtsdf;

namespace dbtsdf {

static thread_local std::string g_err;

// A roctx range over an entry point's host work (rocprofv3 --marker-trace
// shows it beside the kernels it enqueued).
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};
void set_error(const std::string &msg) { g_err = msg; }

dbtsdf_status check_hip(hipError_t e, const char *what, dbtsdf_grid *g) {
    if (e == hipSuccess) return DBTSDF_OK;
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    (void)hipGetLastError();
    if (e == hipErrorOutOfMemory) return DBTSDF_ERR_OUT_OF_MEMORY;
    if (g) g->poisoned = true;
    return DBTSDF_ERR_DEVICE;
}

static dbtsdf_status invalid(const std::string &msg) {
    set_error(msg);
    return DBTSDF_ERR_INVALID_ARG;
}

static uint32_t next_pow2(uint64_t v, uint32_t lo) {
    uint64_t p = lo;
    while (p < v) p <<= 1;
    return (uint32_t)p;
}

// ------------------------------------------------------------- tables ---
DeviceTables::~DeviceTables() {
    for (void *p : allocs) (void)hipFree(p);
}

template <typename T>
static hipError_t upload(DeviceTables &d, const std::vector<T> &v, const T **out) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(1, v.size()) * sizeof(T));
    if (e != hipSuccess) return e;
    d.allocs.push_back(p);
    if (!v.empty()) e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    *out = (const T *)p;
    return e;
}

static dbtsdf_status make_device_tables(const KernelSet &ks, std::shared_ptr<DeviceTables> &out) {
    auto d = std::make_shared<DeviceTables>();
    d->params = ks.p;
    for (size_t b = 0; b + 1 < ks.sh_start.size(); ++b)
        d->max_shadow = std::max(d->max_shadow, ks.sh_start[b + 1] - ks.sh_start[b]);
    DevTables &t = d->t;
    hipError_t e = upload(*d, ks.mask_by_q, &t.mask_by_q);
    if (e == hipSuccess) e = upload(*d, ks.sh_start, &t.sh_start);
    if (e == hipSuccess) e = upload(*d, ks.sh_off, &t.sh_off);
    if (e == hipSuccess) e = upload(*d, ks.az_c, &t.az_c);
    if (e == hipSuccess) e = upload(*d, ks.az_s, &t.az_s);
    if (e == hipSuccess) e = upload(*d, ks.el_s2, &t.el_s2);
    if (e == hipSuccess) e = upload(*d, ks.el_neg, &t.el_neg);
    t.row_image = nullptr;
    if (e == hipSuccess && !ks.row_image.empty()) {
        const uint32_t *img = nullptr;
        e = upload(*d, ks.row_image, &img);
        t.row_image = reinterpret_cast<const uint4 *>(img);
    }
    if (e != hipSuccess) return check_hip(e, "uploading kernel tables");
    t.n_q = (uint32_t)ks.mask_by_q.size();
    t.n_bins = ks.n_bins;
    t.K = ks.K;
    t.R = ks.R;
    t.shadow_r2 = ks.p.shadow_r2;
    t.binning = ks.p.binning;
    t.bins_az = ks.p.bins_az;
    t.bins_el = ks.p.bins_el;
    t.metric = ks.p.metric;
    t.shadow_model = ks.p.shadow_model;
    out = std::move(d);
    return DBTSDF_OK;
}

// ---------------------------------------------------------- workspace ---
Workspace::~Workspace() {
    release();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
}

// The graph of (call layout, tuning, capacity, part), captured on the
// workspace's private stream the first time and replayed after that. Kernel
// arguments are baked into the graph; everything that changes from call to
// call (poses, point counts, scans) is read by the kernels from the
// descriptor buffer, uploaded before each launch.
static hipError_t pipeline_graph(Workspace &ws, const PipeArgs &a, const Tuning &tun, int part,
                                 hipGraphExec_t *out) {
    std::string key;
    key.append((const char *)&a, sizeof(a));
    key.append((const char *)&tun, sizeof(tun));
    key.append((const char *)&ws.points_cap, sizeof(ws.points_cap));
    key.append((const char *)&part, sizeof(part));
    auto it = ws.graphs.find(key);
    if (it != ws.graphs.end()) {
        *out = it->second.exec;
        return hipSuccess;
    }
    hipError_t e = hipSuccess;
    if (!ws.cap_stream) e = hipStreamCreateWithFlags(&ws.cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(ws.cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t le = launch_pipeline(a, tun, ws.points_cap, ws.cap_stream, part);
    e = hipStreamEndCapture(ws.cap_stream, &graph);
    if (e == hipSuccess) e = le;
    GraphEntry ge;
    if (e == hipSuccess) e = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    ws.graphs.emplace(key, ge);
    ++ws.captures;
    *out = ge.exec;
    return hipSuccess;
}

void Workspace::drop_graphs() {
    for (auto &kv : graphs)
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    graphs.clear();
}

void Workspace::release() {
    drop_graphs();
    free_sort_buffers(sorter);
    void *ptrs[] = {d_desc, rec, pslot, hkeys, hvals, items, item_off, item_cnt, entries, ctr, staging, rank, work};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    d_desc = nullptr;
    rec = nullptr;
    pslot = nullptr;
    hkeys = nullptr;
    hvals = nullptr;
    items = nullptr;
    item_off = item_cnt = rank = nullptr;
    entries = nullptr;
    work = nullptr;
    ctr = nullptr;
    staging = nullptr;
    staging_cap = 0;
    points_cap = scans_cap = grids_cap = items_cap = entries_cap = hash_cap = 0;
    for (RingSlot &s : ring) {
        if (s.busy && s.ev) (void)hipEventSynchronize(s.ev);
        deliver(s);
        if (s.host) (void)hipHostFree(s.host);
        if (s.ev) (void)hipEventDestroy(s.ev);
        for (hipEvent_t &e : s.pe)
            if (e) (void)hipEventDestroy(e);
    }
    ring.clear();
}

hipError_t Workspace::ensure(uint32_t n_points, uint32_t n_scans, uint32_t n_grids, uint32_t entry_factor,
                             hipStream_t st) {
    const uint64_t need_items = (uint64_t)entry_factor * std::max<uint32_t>(n_points, 1);
    if (n_points <= points_cap && n_scans <= scans_cap && n_grids <= grids_cap && need_items <= items_cap &&
        d_desc)
        return hipSuccess;
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    deliver_all();
    // keep the staging buffer, drop the rest
    float *keep = staging;
    size_t keep_cap = staging_cap;
    staging = nullptr;
    std::vector<RingSlot> keep_ring;
    keep_ring.swap(ring);
    release();
    ring.swap(keep_ring);
    staging = keep;
    staging_cap = keep_cap;

    points_cap = std::max(next_pow2(n_points, 4096), points_cap);
    scans_cap = std::max(next_pow2(n_scans, 16), scans_cap);
    grids_cap = std::max(next_pow2(n_grids, 16), grids_cap);
    const uint64_t ic = (uint64_t)entry_factor * points_cap;
    if (ic > 0xFFFFFFF0ull) return hipErrorInvalidValue;
    items_cap = entries_cap = (uint32_t)ic;
    // a sparse table keeps linear probing short: a wavefront's insert costs as
    // many atomic round trips as its longest probe sequence (load <= 1/8 up to
    // 2^21 points, never above 1/2)
    hash_cap = next_pow2(std::max<uint64_t>(2ull * points_cap, std::min<uint64_t>(8ull * points_cap, 1ull << 24)), 8192);
    desc_bytes = sizeof(Ctrl) + sizeof(CallInfo) + (size_t)grids_cap * sizeof(DevGrid) + (size_t)scans_cap * sizeof(DevScan);
    const size_t ctr_words = (size_t)scans_cap * SC_N + (size_t)grids_cap * TC_N;
    struct A {
        void **p;
        size_t bytes;
    } al[] = {
        {&d_desc, desc_bytes},
        {(void **)&rec, (size_t)points_cap * sizeof(uint4)},
        {(void **)&pslot, (size_t)points_cap * 4},
        {(void **)&hkeys, (size_t)hash_cap * 8},
        {(void **)&hvals, (size_t)hash_cap * 4},
        {(void **)&items, (size_t)items_cap * 8},
        {(void **)&item_off, (size_t)items_cap * 4},
        {(void **)&item_cnt, (size_t)items_cap * 4},
        {(void **)&entries, (size_t)entries_cap * sizeof(uint4)},
        {(void **)&rank, (size_t)entries_cap * 4},
        {(void **)&work, ((size_t)items_cap + entries_cap) * sizeof(uint4)},
        {(void **)&ctr, ctr_words * 8},
    };
    for (auto &a : al) {
        e = hipMalloc(a.p, a.bytes);
        if (e != hipSuccess) {
            release();
            return e;
        }
    }
    e = launch_fill_u64(hkeys, kHashEmpty, hash_cap, st);
    if (e == hipSuccess) e = launch_fill_u32(hvals, 0xFFFFFFFFu, hash_cap, st);
    if (e == hipSuccess) e = hipMemsetAsync(d_desc, 0, desc_bytes, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

hipError_t Workspace::ensure_staging(size_t floats, hipStream_t st) {
    if (floats <= staging_cap && staging) return hipSuccess;
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    if (staging) (void)hipFree(staging);
    staging = nullptr;
    size_t cap = std::max<size_t>(floats, 3 * 4096);
    cap = std::max(cap, staging_cap * 2);
    e = hipMalloc((void **)&staging, cap * sizeof(float));
    staging_cap = e == hipSuccess ? cap : 0;
    drop_graphs();
    return e;
}

static_assert(sizeof(Ctrl) % 8 == 0 && sizeof(CallInfo) % 8 == 0 && sizeof(DevGrid) % 8 == 0 &&
                  sizeof(DevScan) % 8 == 0,
              "descriptors are copied in 8-byte words");

// A ring slot's buffer: pinned, coherent host memory that the first and last
// passes of a call read and write directly.
static bool alloc_slot(RingSlot &r, size_t bytes) {
    if (hipHostMalloc(&r.host, bytes, hipHostMallocCoherent) != hipSuccess) {
        (void)hipGetLastError();
        r.host = nullptr;
        return false;
    }
    if (hipHostGetDevicePointer(&r.host_dev, r.host, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(r.host);
        r.host = r.host_dev = nullptr;
        return false;
    }
    r.bytes = bytes;
    return true;
}

RingSlot &Workspace::next_slot(size_t bytes, std::string *err) {
    constexpr uint32_t kRing = 16;
    if (ring.size() < kRing) {
        // allocate every slot up front: pinned allocations are slow and must
        // not land in the middle of a run of calls
        ring.resize(kRing);
        for (RingSlot &r : ring) {
            if (!r.ev) (void)hipEventCreateWithFlags(&r.ev, hipEventDisableTiming);
            for (hipEvent_t &e : r.pe)
                if (!e) (void)hipEventCreate(&e);
            const size_t want = std::max<size_t>(bytes, 64 * 1024);
            if (!r.host) alloc_slot(r, want);
        }
    }
    RingSlot &s = ring[ring_next];
    ring_next = (ring_next + 1) % kRing;
    if (s.busy) {
        (void)hipEventSynchronize(s.ev);
        deliver(s);
    }
    if (s.bytes < bytes) {
        if (s.host) (void)hipHostFree(s.host);
        s.host = s.host_dev = nullptr;
        s.bytes = 0;
        drop_graphs();  // graphs bake the slot's address in
        if (!alloc_slot(s, bytes) && err) *err = "pinned descriptor allocation failed";
    }
    return s;
}

void Workspace::deliver(RingSlot &s) {
    if (!s.busy) return;
    const unsigned long long *c = (const unsigned long long *)((const char *)s.host + s.ctr_off);
    for (const PendingStat &p : s.pend) {
        dbtsdf_scan_stats st{};
        const unsigned long long *sc = c + (size_t)p.scan * SC_N;
        st.n_in = p.n_in;
        st.n_invalid = sc[SC_INVALID];
        st.n_out_of_bounds = sc[SC_OOB];
        st.n_duplicate = sc[SC_DUP];
        st.n_integrated = sc[SC_INT];
        st.voxel_updates = sc[SC_INT] * p.k3;
        st.shadow_updates = sc[SC_SHADOW];
        st.n_revisit = sc[SC_REVISIT];
        if (p.traffic_grid >= 0) {
            const unsigned long long *tc = c + (size_t)scans_cap * SC_N + (size_t)p.traffic_grid * TC_N;
            st.u_mask = tc[TC_UMASK];
            st.c_mask = tc[TC_CMASK];
            st.u_shadow = tc[TC_USHADOW];
        }
        if (p.dst) *p.dst = st;
    }
    s.pend.clear();
    if (s.prof) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, s.pe[0], s.pe[2]) == hipSuccess) {
            prof_call_ms += ms;
            ++prof_calls;
        }
        if (s.prof == 2 && hipEventElapsedTime(&ms, s.pe[1], s.pe[2]) == hipSuccess) {
            prof_apply_ms += ms;
            ++prof_apply;
        }
        s.prof = 0;
    }
    s.busy = false;
}

void Workspace::deliver_all() {
    for (RingSlot &s : ring) {
        if (!s.busy) continue;
        (void)hipEventSynchronize(s.ev);
        deliver(s);
    }
}

// ------------------------------------------------------------ bricks ---
dbtsdf_status ensure_bricks(dbtsdf_grid *g) {
    const Tuning &t = g->tuning;
    if (g->brick_cnt && g->brick_dims[0] == t.bx && g->brick_dims[1] == t.by && g->brick_dims[2] == t.bz)
        return DBTSDF_OK;
    hipError_t e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return check_hip(e, "synchronising before brick re-allocation", g);
    if (g->brick_cnt) (void)hipFree(g->brick_cnt);
    if (g->brick_slot) (void)hipFree(g->brick_slot);
    g->brick_cnt = g->brick_slot = nullptr;
    const uint32_t bd[3] = {t.bx, t.by, t.bz};
    uint64_t nbr = 1;
    for (int k = 0; k < 3; ++k) {
        g->nb[k] = (g->params.dims[k] + bd[k] - 1) / bd[k];
        nbr *= g->nb[k];
        g->brick_dims[k] = bd[k];
    }
    // a power of two of counters: the tile strategy indexes them through a
    // multiplicative bijection on that range
    uint64_t cap = 1;
    while (cap < nbr) cap <<= 1;
    e = hipMalloc((void **)&g->brick_cnt, cap * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&g->brick_slot, cap * 4);
    if (e == hipSuccess) e = launch_fill_u32(g->brick_cnt, 0u, cap, g->stream);
    if (e != hipSuccess) {
        g->brick_cnt = nullptr;
        return check_hip(e, "allocating brick counters", g);
    }
    if (g->ws) g->ws->drop_graphs();
    return DBTSDF_OK;
}

static uint32_t entry_factor(const Tuning &t, int R) {
    const uint32_t b[3] = {t.bx, t.by, t.bz};
    uint32_t f = 1;
    for (int k = 0; k < 3; ++k) f *= 1u + (2u * R + b[k] - 1u) / b[k];
    return f;
}

// ------------------------------------------------------------ enqueue ---
DevGrid dev_grid_of(const dbtsdf_grid *g, uint32_t index) {
    DevGrid d{};
    d.mask = g->mask;
    d.packed = g->packed;
    d.brick_cnt = g->brick_cnt;
    d.brick_slot = g->brick_slot;
    d.nx = g->params.dims[0];
    d.ny = g->params.dims[1];
    d.nz = g->params.dims[2];
    d.nbx = g->nb[0];
    d.nby = g->nb[1];
    d.nbz = g->nb[2];
    d.T = g->params.hit_threshold;
    d.hmax = g->params.hit_max;
    d.traffic_slot = index;
    d.revisit_skip = g->revisit_skip ? 1u : 0u;
    return d;
}

DevScan dev_scan_of(const ScanIn &s, uint32_t begin, uint32_t grid_index) {
    const dbtsdf_grid_params &gp = s.grid->params;
    DevScan d{};
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) d.rot[3 * r + c] = s.pose[4 * r + c];
        d.trans[r] = s.pose[4 * r + 3];
        d.origin[r] = gp.origin[r];
    }
    d.inv_s = 1.0f / gp.voxel_size;
    d.pts = s.points;
    d.begin = begin;
    d.n = (uint32_t)s.n;
    d.grid = grid_index;
    d.dedup = (gp.flags & DBTSDF_DEDUP_FIRST) ? 1u : 0u;
    d.step = s.step;
    if (s.times) {
        d.deskew = 1;
        d.times = s.times;
        for (int k = 0; k < 4; ++k) d.dq[k] = s.dq[k];
        for (int k = 0; k < 3; ++k) d.dt[k] = s.dt[k];
    }
    return d;
}

// The per-point strategy's row kernel covers a call when the kernel set has
// its tables and every grid has 16-byte aligned rows and window byte offsets
// within 32 bits.
bool row_kernel_tables(const dbtsdf_grid *g) { return g->tables->t.row_image != nullptr; }

bool row_kernel_covers(const dbtsdf_grid *g) {
    if (g->tables->t.row_image == nullptr) return false;
    const uint64_t span = (uint64_t)g->tables->t.R *
                          (1ull + g->params.dims[0] + (uint64_t)g->params.dims[0] * g->params.dims[1]);
    return g->params.dims[0] % 4u == 0 && 8 * span < (1ull << 32);
}


dbtsdf_status enqueue_scans(Workspace &ws, hipStream_t st, std::vector<ScanIn> &scans, bool use_graph, bool plain) {
    // drop empty scans (their statistics are all zero)
    std::vector<ScanIn> live;
    for (ScanIn &s : scans) {
        if (s.n == 0) {
            if (s.stats) *s.stats = dbtsdf_scan_stats{};
        } else {
            live.push_back(s);
        }
    }
    if (live.empty()) return DBTSDF_OK;
    dbtsdf_grid *g0 = live[0].grid;
    std::vector<dbtsdf_grid *> grids;
    std::unordered_map<dbtsdf_grid *, uint32_t> gidx;
    uint64_t total = 0;
    bool traffic = false;
    for (ScanIn &s : live) {
        dbtsdf_grid *g = s.grid;
        if (g->poisoned) {
            set_error("grid is poisoned by an earlier device error");
            return DBTSDF_ERR_POISONED;
        }
        if (g->device != g0->device) return invalid("all grids of a batch must be on one device");
        if (std::memcmp(&g->kparams, &g0->kparams, sizeof(g->kparams)) != 0)
            return invalid("all grids of a batch must share the kernel parameters");
        if (g->tuning.strategy != g0->tuning.strategy || g->tuning.bx != g0->tuning.bx ||
            g->tuning.by != g0->tuning.by || g->tuning.bz != g0->tuning.bz || g->tuning.threads != g0->tuning.threads)
            return invalid("all grids of a batch must share the tuning");
        if (!gidx.count(g)) {
            gidx[g] = (uint32_t)grids.size();
            grids.push_back(g);
        }
        traffic |= (g->params.flags & DBTSDF_COUNT_TRAFFIC) != 0;
        total += s.n;
    }
    if (total > kMaxPointsPerCall) {
        set_error("too many points in one call");
        return DBTSDF_ERR_OUT_OF_RANGE;
    }
    if (live.size() > kMaxScansPerCall) {
        set_error("too many scans in one call");
        return DBTSDF_ERR_OUT_OF_RANGE;
    }
    Tuning tun = g0->tuning;
    if (traffic) tun.strategy = DBTSDF_STRATEGY_BRICK;  // unique-word counts come from the brick merge
    // the per-point strategy carries a survivor's grid in 16 bits
    if (grids.size() > kMaxAtomicGrids) tun.strategy = DBTSDF_STRATEGY_BRICK;
    // the per-point strategy's row kernel: tables for the kernel set, 16-byte
    // aligned grid rows and window byte offsets within 32 bits in every grid
    bool row_kernel = true;
    for (dbtsdf_grid *g : grids) row_kernel = row_kernel && row_kernel_covers(g);
    if (tun.apply_blocks == 0) tun.apply_blocks = (uint32_t)apply_blocks_default(tun, g0->K, row_kernel, g0->device);
    for (dbtsdf_grid *g : grids) {
        dbtsdf_status s = ensure_bricks(g);
        if (s != DBTSDF_OK) return s;
    }
    const int R = g0->tables->t.R;
    const uint32_t ef = entry_factor(tun, R);
    hipError_t e = ws.ensure((uint32_t)total, (uint32_t)live.size(), (uint32_t)grids.size(), ef, st);
    if (e != hipSuccess) return check_hip(e, "allocating the workspace", g0);

    // descriptors, laid out as on the device: CallInfo | DevGrid[grids_cap] | DevScan[n_scans]
    const size_t n_sc = live.size(), n_gr = grids.size();
    const size_t scans_off = sizeof(CallInfo) + (size_t)ws.grids_cap * sizeof(DevGrid);
    const size_t ctr_bytes = ((size_t)ws.scans_cap * SC_N + (size_t)ws.grids_cap * TC_N) * 8;
    // counters at a fixed place in the slot (a captured graph bakes the address in)
    const size_t ctr_off = (scans_off + (size_t)ws.scans_cap * sizeof(DevScan) + 255) & ~(size_t)255;
    std::string err;
    RingSlot &slot = ws.next_slot(ctr_off + ctr_bytes, &err);
    if (!slot.host) {
        set_error(err);
        return DBTSDF_ERR_OUT_OF_MEMORY;
    }
    char *h = (char *)slot.host;
    CallInfo ci{(uint32_t)total, (uint32_t)n_sc, (uint32_t)n_gr, 0};
    std::memcpy(h, &ci, sizeof(ci));
    DevGrid *hg = (DevGrid *)(h + sizeof(CallInfo));
    for (size_t i = 0; i < n_gr; ++i) {
        const DevGrid d = dev_grid_of(grids[i], (uint32_t)i);
        std::memcpy(&hg[i], &d, sizeof(d));
    }
    DevScan *hs = (DevScan *)(h + scans_off);
    uint32_t begin = 0;
    std::vector<bool> traffic_given(n_gr, false);
    slot.pend.clear();
    const uint64_t k3 = (uint64_t)g0->K * g0->K * g0->K;
    for (size_t i = 0; i < n_sc; ++i) {
        const ScanIn &s = live[i];
        const dbtsdf_grid_params &gp = s.grid->params;
        const DevScan d = dev_scan_of(s, begin, gidx[s.grid]);
        std::memcpy(&hs[i], &d, sizeof(d));
        begin += (uint32_t)s.n;
        PendingStat p{s.stats, (uint32_t)i, -1, s.n, k3};
        if ((gp.flags & DBTSDF_COUNT_TRAFFIC) && !traffic_given[d.grid]) {
            p.traffic_grid = (int32_t)d.grid;
            traffic_given[d.grid] = true;
        }
        if (s.stats) slot.pend.push_back(p);
    }
    char *dd = (char *)ws.d_desc;

    PipeArgs a{};
    a.ctrl = (Ctrl *)dd;
    a.grids = (const DevGrid *)(dd + sizeof(Ctrl) + sizeof(CallInfo));
    a.scans = (const DevScan *)(dd + sizeof(Ctrl) + scans_off);
    a.tab = g0->tables->t;
    a.brick[0] = tun.bx;
    a.brick[1] = tun.by;
    a.brick[2] = tun.bz;
    a.hash_mask = ws.hash_cap - 1;
    a.rec = ws.rec;
    a.pslot = ws.pslot;
    a.hkeys = ws.hkeys;
    a.hvals = ws.hvals;
    a.items = ws.items;
    a.item_off = ws.item_off;
    a.item_cnt = ws.item_cnt;
    a.rank = ws.rank;
    a.work = ws.work;
    a.entries = ws.entries;
    a.surv_rec = ws.entries;  // the brick lists' storage (at least one uint4 per point)
    a.host_desc = (const uint2 *)slot.host_dev;
    a.host_ctr = (unsigned long long *)((char *)slot.host_dev + ctr_off);
    a.desc_scans_off = (uint32_t)scans_off;
    a.scans_cap = ws.scans_cap;
    a.scan_ctr = ws.ctr;
    a.traffic_ctr = ws.ctr + (size_t)ws.scans_cap * SC_N;
    a.items_cap = ws.items_cap;
    a.entries_cap = ws.entries_cap;
    a.count_traffic = traffic ? 1u : 0u;
    {
        const uint32_t bd[3] = {tun.bx, tun.by, tun.bz};
        for (int k = 0; k < 3; ++k) a.span[k] = 1u + (2u * (uint32_t)R + bd[k] - 1u) / bd[k];
    }
    // exact unique-word counts need every brick merged by one work unit; the
    // tile strategy never splits a tile
    a.chunk = traffic || tun.strategy == DBTSDF_STRATEGY_TILE ? 0u : tun.chunk;
    // the plain one-scan call has a kernel of its own (no per-point scan lookup)
    // (its front pass reads the scan descriptor from the host in 16-byte pieces)
    a.single_scan = plain && live.size() == 1 && scans_off % 16 == 0 ? 1u : 0u;
    a.row_kernel = row_kernel ? 1u : 0u;
    a.revisit_ok = g0->tables->t.n_bins <= 32768u ? 1u : 0u;
    a.tile_mode = tun.strategy == DBTSDF_STRATEGY_TILE ? 1u : 0u;
    if (a.tile_mode && !row_kernel_tables(g0)) return invalid("the tile strategy needs K <= 11, at most 31 bins and r_s^2 <= 9");

    // batches that ask for it, and plain brick-strategy calls (nine passes),
    // replay captured graphs (one host call instead of one per pass); plain
    // per-point calls launch their three passes directly, which measured
    // faster than a graph launch; with profiling on, events bracket the call
    // and its apply kernel
    // (the sort strategy reads counts back in the middle of its apply and
    // launches directly)
    const bool sort = tun.strategy == DBTSDF_STRATEGY_SORT;
    const bool graphs = !sort && (use_graph || (plain && tun.strategy == DBTSDF_STRATEGY_BRICK));
    SortPlan plan{};
    if (sort) {
        uint64_t max_vox = 0;
        for (dbtsdf_grid *g : grids) max_vox = std::max<uint64_t>(max_vox, g->n_voxels);
        while ((1ull << plan.shift) < max_vox) ++plan.shift;
        uint32_t gbits = 0;
        while ((1ull << gbits) < grids.size()) ++gbits;
        plan.end_bit = plan.shift + gbits;
        if (plan.end_bit == 0) plan.end_bit = 1;
        plan.emit_blocks = tun.apply_blocks;
        plan.pairs_per_point = k3 + g0->tables->max_shadow;
        const uint32_t K = (uint32_t)g0->K, rows_per_pass = 64u / K;
        plan.words = (K * K + rows_per_pass - 1u) / rows_per_pass + (g0->tables->max_shadow + 63u) / 64u;
        plan.round_survivors = tun.chunk;
    }
    auto apply_part = [&]() -> hipError_t {
        return sort ? sort_apply(ws, a, plan, st) : launch_pipeline(a, tun, ws.points_cap, st, kPartApply);
    };
    slot.prof = 0;
    auto run_part = [&](int part) -> hipError_t {
        if (sort) {
            hipError_t se = hipSuccess;
            if (part == kPartAll || part == kPartPre) se = launch_pipeline(a, tun, ws.points_cap, st, kPartPre);
            if (se == hipSuccess && (part == kPartAll || part == kPartApply)) se = apply_part();
            return se;
        }
        if (!graphs) return launch_pipeline(a, tun, ws.points_cap, st, part);
        hipGraphExec_t ex = nullptr;
        hipError_t ge = pipeline_graph(ws, a, tun, part, &ex);
        if (ge != hipSuccess) return ge;
        ++ws.replays;
        return hipGraphLaunch(ex, st);
    };
    // with profiling on, the calls whose index is a multiple of prof_every
    // are timed (the index runs over all calls, so with a period that
    // divides the ring size a ring slot is always timed or never)
    const uint64_t call_index = ws.n_calls++;
    const bool timed = ws.prof_every && call_index % ws.prof_every == 0;
    if (timed) {
        // the apply kernel is launched directly between its two events, so
        // they time the kernel rather than a graph launch around it
        e = hipEventRecord(slot.pe[0], st);
        if (e == hipSuccess) e = run_part(kPartPre);
        if (e == hipSuccess) e = hipEventRecord(slot.pe[1], st);
        if (e == hipSuccess) e = apply_part();
        if (e == hipSuccess) e = hipEventRecord(slot.pe[2], st);
        if (e == hipSuccess && pipeline_has_post(tun)) e = run_part(kPartPost);
        slot.prof = 2;
    } else {
        e = run_part(kPartAll);
    }
    if (e != hipSuccess) return check_hip(e, "launching the integration kernels", g0);

    slot.ctr_off = ctr_off;
    e = hipEventRecord(slot.ev, st);
    if (e != hipSuccess) return check_hip(e, "queueing statistics readback", g0);
    slot.busy = true;
    return DBTSDF_OK;
}

}  // namespace dbtsdf

// =================================================================== C ABI ===
extern "C" {

const char *dbtsdf_status_string(dbtsdf_status s) {
    switch (s) {
        case DBTSDF_OK: return "ok";
        case DBTSDF_ERR_INVALID_ARG: return "invalid argument";
        case DBTSDF_ERR_OUT_OF_MEMORY: return "out of memory";
        case DBTSDF_ERR_DEVICE: return "device error";
        case DBTSDF_ERR_OUT_OF_RANGE: return "out of range";
        case DBTSDF_ERR_POISONED: return "grid poisoned by an earlier device error";
        case DBTSDF_ERR_BUSY: return "busy";
    }
    return "unknown status";
}

const char *dbtsdf_last_error(void) { return g_err.c_str(); }

uint64_t dbtsdf_now_ns(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

// ------------------------------------------------------------ kernel sets ---
dbtsdf_status dbtsdf_kernel_set_create(const dbtsdf_kernel_params *params, dbtsdf_kernel_set **out) {
    if (!params || !out) return invalid("NULL argument");
    std::string err;
    KernelSet *ks = build_kernel_set(*params, &err);
    if (!ks) return invalid(err);
    *out = new dbtsdf_kernel_set();
    (*out)->ks.reset(ks);
    return DBTSDF_OK;
}

dbtsdf_status dbtsdf_kernel_set_export(const dbtsdf_kernel_set *k, uint32_t *masks, uint8_t *shadow, double *dirs,
                                       uint32_t *n_bins) {
    if (!k || !k->ks) return invalid("NULL kernel set");
    const KernelSet &ks = *k->ks;
    if (masks) std::memcpy(masks, ks.cell_mask.data(), ks.cell_mask.size() * 4);
    if (shadow) std::memcpy(shadow, ks.shadow.data(), ks.shadow.size());
    if (dirs) std::memcpy(dirs, ks.dirs.data(), ks.dirs.size() * 8);
    if (n_bins) *n_bins = ks.n_bins;
    return DBTSDF_OK;
}

uint32_t dbtsdf_kernel_set_n_bins(const dbtsdf_kernel_set *k) { return (k && k->ks) ? k->ks->n_bins : 0; }

int32_t dbtsdf_kernel_set_bin(const dbtsdf_kernel_set *k, float dx, float dy, float dz) {
    if (!k || !k->ks) return -1;
    return host_bin(*k->ks, dx, dy, dz);
}

void dbtsdf_kernel_set_destroy(dbtsdf_kernel_set *k) { delete k; }

// ------------------------------------------------------------------ grids ---
uint64_t dbtsdf_grid_bytes(const dbtsdf_grid_params *p) {
    if (!p) return 0;
    return (uint64_t)p->dims[0] * p->dims[1] * p->dims[2] * 8ull;
}

static dbtsdf_status validate_grid_params(const dbtsdf_grid_params *p, int K) {
    if (!p) return invalid("NULL grid params");
    for (int k = 0; k < 3; ++k) {
        if (p->dims[k] < (uint32_t)K || p->dims[k] > kMaxDim) return invalid("each dim must be in [K, 2^20]");
        if (!std::isfinite(p->origin[k])) return invalid("origin must be finite");
    }
    const uint64_t nv = (uint64_t)p->dims[0] * p->dims[1] * p->dims[2];
    if (nv >= (1ull << kVoxelKeyBits)) return invalid("grid has too many voxels");
    if (!std::isfinite(p->voxel_size) || !(p->voxel_size > 0.0f)) return invalid("voxel_size must be finite and > 0");
    if (!std::isfinite(1.0f / p->voxel_size)) return invalid("voxel_size too small");
    if (p->hit_max < 1 || p->hit_max > 65535) return invalid("hit_max must be in 1..65535");
    if (p->hit_threshold > 65535) return invalid("hit_threshold must be <= 65535");
    if (p->flags & ~(DBTSDF_DEDUP_FIRST | DBTSDF_COUNT_TRAFFIC)) return invalid("unknown grid flags");
    return DBTSDF_OK;
}

static dbtsdf_status create_grid_impl(const dbtsdf_grid_params *params, const dbtsdf_kernel_set *ks, void *stream,
                                      void *mask_dev, void *packed_dev, dbtsdf_grid **out) {
    if (!out) return invalid("NULL out");
    *out = nullptr;
    if (!ks || !ks->ks) return invalid("NULL kernel set");
    dbtsdf_status s = validate_grid_params(params, ks->ks->K);
    if (s != DBTSDF_OK) return s;
    auto g = std::make_unique<dbtsdf_grid>();
    g->params = *params;
    g->kparams = ks->ks->p;
    g->K = ks->ks->K;
    g->stream = (hipStream_t)stream;
    g->n_voxels = (uint64_t)params->dims[0] * params->dims[1] * params->dims[2];
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) return check_hip(e, "hipGetDevice");
    {
        // one device copy of the tables per kernel set and device: grids made
        // from the same kernel set also share their captured graphs
        std::lock_guard<std::mutex> lk(const_cast<dbtsdf_kernel_set *>(ks)->mu);
        auto &slot = const_cast<dbtsdf_kernel_set *>(ks)->dev[g->device];
        if (!slot) {
            s = make_device_tables(*ks->ks, slot);
            if (s != DBTSDF_OK) {
                slot.reset();
                return s;
            }
        }
        g->tables = slot;
    }
    if (mask_dev || packed_dev) {
        if (!mask_dev || !packed_dev) return invalid("both planes must be given");
        if (((uintptr_t)mask_dev | (uintptr_t)packed_dev) & 15u) return invalid("planes must be 16-byte aligned");
        g->owns_planes = false;
        g->mask = (uint32_t *)mask_dev;
        g->packed = (uint32_t *)packed_dev;
    } else {
        e = hipMalloc((void **)&g->mask, g->n_voxels * 4);
        if (e == hipSuccess) e = hipMalloc((void **)&g->packed, g->n_voxels * 4);
        if (e != hipSuccess) {
            if (g->mask) (void)hipFree(g->mask);
            g->mask = nullptr;
            (void)hipGetLastError();
            set_error("grid planes do not fit in device memory");
            return DBTSDF_ERR_OUT_OF_MEMORY;
        }
    }
    e = launch_grid_init(g->mask, g->packed, g->n_voxels, g->stream);
    if (e != hipSuccess) return check_hip(e, "filling the initial state");
    e = hipEventCreateWithFlags(&g->ev, hipEventDisableTiming);
    if (e != hipSuccess) return check_hip(e, "hipEventCreate");
    g->tuning = Tuning{};
    g->ws = std::make_unique<Workspace>();
    g->ws->device = g->device;
    s = ensure_bricks(g.get());
    if (s != DBTSDF_OK) return s;
    *out = g.release();
    return DBTSDF_OK;
}

dbtsdf_status dbtsdf_create_grid(const dbtsdf_grid_params *params, const dbtsdf_kernel_set *ks, void *hip_stream,
                                 dbtsdf_grid **out) {
    return create_grid_impl(params, ks, hip_stream, nullptr, nullptr, out);
}

dbtsdf_status dbtsdf_create_grid_on(const dbtsdf_grid_params *params, const dbtsdf_kernel_set *ks, void *hip_stream,
                                    void *mask_dev, void *packed_dev, dbtsdf_grid **out) {
    if (!mask_dev || !packed_dev) return invalid("NULL plane");
    return create_grid_impl(params, ks, hip_stream, mask_dev, packed_dev, out);
}

dbtsdf_status dbtsdf_grid_planes(const dbtsdf_grid *g, void **mask_dev, void **packed_dev) {
    if (!g) return invalid("NULL grid");
    if (mask_dev) *mask_dev = g->mask;
    if (packed_dev) *packed_dev = g->packed;
    return DBTSDF_OK;
}

dbtsdf_status dbtsdf_reset_grid(dbtsdf_grid *g) {
    if (!g) return invalid("NULL grid");
    if (g->poisoned) return DBTSDF_ERR_POISONED;
    const dbtsdf_status s = check_hip(launch_grid_init(g->mask, g->packed, g->n_voxels, g->stream), "resetting the grid", g);
    if (s == DBTSDF_OK) g->revisit_skip = true;
    return s;
}

dbtsdf_status dbtsdf_get_tuning(const dbtsdf_grid *g, dbtsdf_tuning *out) {
    if (!g || !out) return invalid("NULL argument");
    out->strategy = g->tuning.strategy;
    out->brick[0] = g->tuning.bx;
    out->brick[1] = g->tuning.by;
    out->brick[2] = g->tuning.bz;
    out->block_threads = g->tuning.threads;
    out->apply_blocks = g->tuning.apply_blocks;
    out->chunk = g->tuning.chunk ? g->tuning.chunk : 0xFFFFFFFFu;
    return DBTSDF_OK;
}

dbtsdf_status dbtsdf_set_tuning(dbtsdf_grid *g, const dbtsdf_tuning *t) {
    if (!g || !t) return invalid("NULL argument");
    Tuning n;
    n.strategy = t->strategy == DBTSDF_STRATEGY_AUTO ? (uint32_t)DBTSDF_STRATEGY_ATOMIC : t->strategy;
    n.bx = t->brick[0];
    n.by = t->brick[1];
    n.bz = t->brick[2];
    n.threads = t->block_threads;
    n.apply_blocks = t->apply_blocks;
    n.chunk = t->chunk == 0 ? Tuning{}.chunk : (t->chunk == 0xFFFFFFFFu ? 0u : t->chunk);
    // the sort strategy's chunk: most survivors per round (0: as many as the pair buffers allow)
    if (n.strategy == DBTSDF_STRATEGY_SORT) n.chunk = t->chunk == 0xFFFFFFFFu ? 0u : t->chunk;
    if (n.strategy == DBTSDF_STRATEGY_TILE) {
        if (!row_kernel_tables(g)) return invalid("the tile strategy needs K <= 11, at most 31 bins and r_s^2 <= 9");
        if (n.bx == 0 && n.by == 0 && n.bz == 0) {
            n.bx = kTileX;
            n.by = kTileY;
            n.bz = kTileZ;
        }
        if (n.threads == 0) n.threads = 256;
    }
    if (n.strategy == DBTSDF_STRATEGY_ATOMIC || n.strategy == DBTSDF_STRATEGY_SORT) {
        if (n.bx == 0) {
            n.bx = g->tuning.bx;
            n.by = g->tuning.by;
            n.bz = g->tuning.bz;
        }
        Tuning probe = n;
        probe.strategy = DBTSDF_STRATEGY_BRICK;
        probe.threads = 256;
        if (!tuning_supported(probe, g->K)) return invalid("unsupported brick shape");
        if (n.threads == 0) n.threads = 256;
    }
    if (!tuning_supported(n, g->K)) return invalid("unsupported tuning");
    if (n.apply_blocks > (1u << 20)) return invalid("apply_blocks too large");
    g->tuning = n;
    g->ws->drop_graphs();
    return ensure_bricks(g);
}

dbtsdf_status dbtsdf_integrate_scan(dbtsdf_grid *g, const float pose[16], const float *points, uint64_t n,
                                    int points_on_device, dbtsdf_scan_stats *stats) {
    return dbtsdf_integrate_scan_every(g, pose, points, n, 1, points_on_device, stats);
}

static dbtsdf_status integrate_plain(dbtsdf_grid *g, const float pose[16], const float *pose_end, int mode,
                                     const float *points, const float *times, uint64_t n, uint32_t every,
                                     int points_on_device, dbtsdf_scan_stats *stats) {
    TraceRange trace_range("dbtsdf_integrate_scan");
    if (!g || !pose) return invalid("NULL argument");
    if (every == 0) return invalid("every must be >= 1");
    if (g->poisoned) {
        set_error("grid is poisoned by an earlier device error");
        return DBTSDF_ERR_POISONED;
    }
    for (int k = 0; k < 16; ++k)
        if (!std::isfinite(pose[k])) return invalid("pose must be finite");
    float sweep[7] = {1.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (pose_end) {
        if (!times) return invalid("NULL times");
        if (!sweep_constants(pose, pose_end, mode, sweep)) return invalid("non-finite end pose or unknown deskew mode");
    }
    if (n > kMaxPointsPerCall) {
        set_error("too many points in one call");
        return DBTSDF_ERR_OUT_OF_RANGE;
    }
    if (n && !points) return invalid("NULL points");
    if (n == 0) {
        if (stats) *stats = dbtsdf_scan_stats{};
        return DBTSDF_OK;
    }
    const float *dev = points, *dev_t = times;
    if (!points_on_device) {
        // points, then the time fractions, in one staging buffer
        const size_t floats = pose_end ? 4 * n : 3 * n;
        hipError_t e = g->ws->ensure_staging(floats, g->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(g->ws->staging, points, 12 * n, hipMemcpyHostToDevice, g->stream);
        if (e == hipSuccess && pose_end)
            e = hipMemcpyAsync(g->ws->staging + 3 * n, times, 4 * n, hipMemcpyHostToDevice, g->stream);
        if (e != hipSuccess) return check_hip(e, "staging host points", g);
        dev = g->ws->staging;
        dev_t = pose_end ? g->ws->staging + 3 * n : nullptr;
    }
    ScanIn in{g, pose, dev, (n + every - 1) / every, stats, every};
    if (pose_end) {
        in.times = dev_t;
        for (int k = 0; k < 4; ++k) in.dq[k] = sweep[k];
        for (int k = 0; k < 3; ++k) in.dt[k] = sweep[4 + k];
    }
    std::vector<ScanIn> v{in};
    return enqueue_scans(*g->ws, g->stream, v, false, true);
}

dbtsdf_status dbtsdf_integrate_scan_every(dbtsdf_grid *g, const float pose[16], const float *points, uint64_t n,
                                          uint32_t every, int points_on_device, dbtsdf_scan_stats *stats) {
    return integrate_plain(g, pose, nullptr, 0, points, nullptr, n, every, points_on_device, stats);
}

dbtsdf_status dbtsdf_integrate_scan_deskew(dbtsdf_grid *g, const float pose_start[16], const float pose_end[16],
                                           const float *points, const float *times, uint64_t n, uint32_t every,
                                           int mode, int points_on_device, dbtsdf_scan_stats *stats) {
    if (!pose_end) return invalid("NULL argument");
    return integrate_plain(g, pose_start, pose_end, mode, points, times, n, every, points_on_device, stats);
}

dbtsdf_status dbtsdf_sync(dbtsdf_grid *g) {
    TraceRange trace_range("dbtsdf_sync");
    if (!g) return invalid("NULL grid");
    if (g->poisoned) return DBTSDF_ERR_POISONED;
    hipError_t e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return check_hip(e, "synchronising the grid stream", g);
    g->ws->deliver_all();
    return DBTSDF_OK;
}

static dbtsdf_status check_box(const dbtsdf_grid *g, const uint32_t lo[3], const uint32_t hi[3]) {
    if (!g || !lo || !hi) return invalid("NULL argument");
    for (int k = 0; k < 3; ++k)
        if (lo[k] >= hi[k] || hi[k] > g->params.dims[k]) {
            set_error("box must satisfy lo < hi <= dims");
            return DBTSDF_ERR_OUT_OF_RANGE;
        }
    return DBTSDF_OK;
}

static dbtsdf_status gather(dbtsdf_grid *g, const uint32_t lo[3], const uint32_t hi[3], const uint32_t *plane,
                            const uint32_t *packed, void *host, size_t elem) {
    const uint64_t n = (uint64_t)(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
    void *tmp = nullptr;
    hipError_t e = hipMalloc(&tmp, n * elem);
    if (e != hipSuccess) return check_hip(e, "readout buffer");
    e = launch_gather_box(plane, packed, g->params.dims, lo, hi, tmp, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e == hipSuccess) e = hipMemcpy(host, tmp, n * elem, hipMemcpyDeviceToHost);
    (void)hipFree(tmp);
    return check_hip(e, "reading voxels", g);
}

dbtsdf_status dbtsdf_read_voxels(dbtsdf_grid *g, const uint32_t lo[3], const uint32_t hi[3], uint32_t *mask_out,
                                 uint32_t *packed_out) {
    TraceRange trace_range("dbtsdf_read_voxels");
    dbtsdf_status s = check_box(g, lo, hi);
    if (s != DBTSDF_OK) return s;
    if (g->poisoned) return DBTSDF_ERR_POISONED;
    if (mask_out && (s = gather(g, lo, hi, g->mask, nullptr, mask_out, 4)) != DBTSDF_OK) return s;
    if (packed_out && (s = gather(g, lo, hi, g->packed, nullptr, packed_out, 4)) != DBTSDF_OK) return s;
    return DBTSDF_OK;
}

dbtsdf_status dbtsdf_read_distance(dbtsdf_grid *g, const uint32_t lo[3], const uint32_t hi[3], int8_t *dist_out) {
    dbtsdf_status s = check_box(g, lo, hi);
    if (s != DBTSDF_OK) return s;
    if (!dist_out) return invalid("NULL output");
    if (g->poisoned) return DBTSDF_ERR_POISONED;
    return gather(g, lo, hi, g->mask, g->packed, dist_out, 1);
}

dbtsdf_status dbtsdf_extract_mesh(dbtsdf_grid *g, const uint32_t lo[3], const uint32_t hi[3], float *tris_dev,
                                  uint64_t max_tris, uint64_t *n_tris) {
    TraceRange trace_range("dbtsdf_extract_mesh");
    if (!g || !n_tris) return invalid("NULL argument");
    if (!tris_dev && max_tris) return invalid("NULL triangle buffer with max_tris > 0");
    *n_tris = 0;
    const uint32_t zero[3] = {0, 0, 0};
    if (!lo != !hi) return invalid("give both box corners or neither");
    if (!lo) {
        lo = zero;
        hi = g->params.dims;
    }
    dbtsdf_status s = check_box(g, lo, hi);
    if (s != DBTSDF_OK) return s;
    if (g->poisoned) return DBTSDF_ERR_POISONED;
    if (hi[0] - lo[0] < 2 || hi[1] - lo[1] < 2 || hi[2] - lo[2] < 2) return DBTSDF_OK;  // no whole cube
    hipError_t e = hipSetDevice(g->device);
    if (e == hipSuccess && !g->mesh_table) {
        e = hipMalloc((void **)&g->mesh_table, sizeof(MeshTable));
        if (e == hipSuccess) e = hipMemcpy(g->mesh_table, &mesh_table(), sizeof(MeshTable), hipMemcpyHostToDevice);
        if (e != hipSuccess && g->mesh_table) {
            (void)hipFree(g->mesh_table);
            g->mesh_table = nullptr;
        }
    }
    if (e == hipSuccess && !g->mesh_count) e = hipMalloc((void **)&g->mesh_count, sizeof(unsigned long long));
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        set_error("mesh export buffers do not fit in device memory");
        return DBTSDF_ERR_OUT_OF_MEMORY;
    }
    MeshArgs m{};
    m.mask = g->mask;
    m.packed = g->packed;
    m.table = g->mesh_table;
    m.out = max_tris ? tris_dev : nullptr;
    m.count = g->mesh_count;
    m.cap = max_tris;
    m.nx = g->params.dims[0];
    m.ny = g->params.dims[1];
    for (int k = 0; k < 3; ++k) {
        m.lo[k] = lo[k];
        m.nc[k] = hi[k] - lo[k] - 1;
        m.origin[k] = g->params.origin[k];
    }
    m.s = g->params.voxel_size;
    unsigned long long count = 0;
    if (e == hipSuccess) e = launch_fill_u64(g->mesh_count, 0ull, 1, g->stream);
    if (e == hipSuccess) e = launch_mesh(m, g->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&count, g->mesh_count, sizeof(count), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return check_hip(e, "extracting the mesh", g);
    *n_tris = count;
    return DBTSDF_OK;
}

dbtsdf_status dbtsdf_extract_points(dbtsdf_grid *g, const uint32_t lo[3], const uint32_t hi[3], float *xyz_dev,
                                    uint64_t max_points, uint64_t *n_points) {
    TraceRange trace_range("dbtsdf_extract_points");
    if (!g || !n_points) return invalid("NULL argument");
    if (!xyz_dev && max_points) return invalid("NULL point buffer with max_points > 0");
    *n_points = 0;
    const uint32_t zero[3] = {0, 0, 0};
    if (!lo != !hi) return invalid("give both box corners or neither");
    if (!lo) {
        lo = zero;
        hi = g->params.dims;
    }
    dbtsdf_status s = check_box(g, lo, hi);
    if (s != DBTSDF_OK) return s;
    if (g->poisoned) return DBTSDF_ERR_POISONED;
    hipError_t e = hipSetDevice(g->device);
    if (e == hipSuccess && !g->mesh_count) e = hipMalloc((void **)&g->mesh_count, sizeof(unsigned long long));
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        set_error("point export counter does not fit in device memory");
        return DBTSDF_ERR_OUT_OF_MEMORY;
    }
    MeshArgs m{};
    m.mask = g->mask;
    m.packed = g->packed;
    m.out = max_points ? xyz_dev : nullptr;
    m.count = g->mesh_count;
    m.cap = max_points;
    m.nx = g->params.dims[0];
    m.ny = g->params.dims[1];
    for (int k = 0; k < 3; ++k) {
        m.lo[k] = lo[k];
        m.nc[k] = hi[k] - lo[k];
        m.origin[k] = g->params.origin[k];
    }
    m.s = g->params.voxel_size;
    unsigned long long count = 0;
    if (e == hipSuccess) e = launch_fill_u64(g->mesh_count, 0ull, 1, g->stream);
    if (e == hipSuccess) e = launch_points(m, g->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&count, g->mesh_count, sizeof(count), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return check_hip(e, "extracting points", g);
    *n_points = count;
    return DBTSDF_OK;
}

dbtsdf_status dbtsdf_write_voxels(dbtsdf_grid *g, const uint32_t *mask_in, const uint32_t *packed_in) {
    if (!g || !mask_in || !packed_in) return invalid("NULL argument");
    if (g->poisoned) return DBTSDF_ERR_POISONED;
    const uint32_t T = g->params.hit_threshold, H = g->params.hit_max;
    const bool can_flip = T >= 1 && T <= H;
    for (uint64_t i = 0; i < g->n_voxels; ++i) {
        const uint32_t m = mask_in[i], p = packed_in[i];
        const uint32_t h = p & 0xFFFFu;
        const bool occupied = (p >> 31) == 0;
        if ((m & (m + 1u)) != 0u) return invalid("mask word is not of the form 2^n - 1");
        if (p & 0x7FFF0000u) return invalid("packed word has bits 16-30 set");
        if (h > H) return invalid("hit counter above hit_max");
        if (occupied != (can_flip && h >= T)) return invalid("sign disagrees with the hit counter");
    }
    hipError_t e = hipStreamSynchronize(g->stream);
    g->revisit_skip = false;  // written planes need not hold whole windows around integrated voxels
    if (e == hipSuccess) e = hipMemcpy(g->mask, mask_in, g->n_voxels * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(g->packed, packed_in, g->n_voxels * 4, hipMemcpyHostToDevice);
    return check_hip(e, "writing voxels", g);
}

void dbtsdf_destroy_grid(dbtsdf_grid *g) {
    if (!g) return;
    (void)hipStreamSynchronize(g->stream);
    g->ws.reset();
    if (g->brick_cnt) (void)hipFree(g->brick_cnt);
    if (g->brick_slot) (void)hipFree(g->brick_slot);
    if (g->owns_planes) {
        if (g->mask) (void)hipFree(g->mask);
        if (g->packed) (void)hipFree(g->packed);
    }
    if (g->ev) (void)hipEventDestroy(g->ev);
    if (g->mesh_table) (void)hipFree(g->mesh_table);
    if (g->mesh_count) (void)hipFree(g->mesh_count);
    delete g;
}

// -------------------------------------------------------------- profiling ---
static dbtsdf_status read_prof(Workspace &ws, hipStream_t st, double *call_ms, uint64_t *calls, double *apply_ms,
                               uint64_t *applies) {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(e, "synchronising for the profile");
    ws.deliver_all();
    if (call_ms) *call_ms = ws.prof_call_ms;
    if (calls) *calls = ws.prof_calls;
    if (apply_ms) *apply_ms = ws.prof_apply_ms;
    if (applies) *applies = ws.prof_apply;
    return DBTSDF_OK;
}

dbtsdf_status dbtsdf_set_profiling(dbtsdf_grid *g, int enable) {
    if (!g) return invalid("NULL grid");
    if (enable < 0) return invalid("negative profiling period");
    g->ws->prof_every = (uint32_t)enable;
    g->ws->prof_call_ms = g->ws->prof_apply_ms = 0.0;
    g->ws->prof_calls = g->ws->prof_apply = 0;
    return DBTSDF_OK;
}

dbtsdf_status dbtsdf_read_profile(dbtsdf_grid *g, double *call_ms, uint64_t *calls, double *apply_ms,
                                  uint64_t *applies) {
    if (!g) return invalid("NULL grid");
    return read_prof(*g->ws, g->stream, call_ms, calls, apply_ms, applies);
}

dbtsdf_status dbtsdf_batch_set_profiling(dbtsdf_batch *b, int enable) {
    if (!b) return invalid("NULL batch");
    if (enable < 0) return invalid("negative profiling period");
    b->ws->prof_every = (uint32_t)enable;
    b->ws->prof_call_ms = b->ws->prof_apply_ms = 0.0;
    b->ws->prof_calls = b->ws->prof_apply = 0;
    return DBTSDF_OK;
}

dbtsdf_status dbtsdf_batch_read_profile(dbtsdf_batch *b, double *call_ms, uint64_t *calls, double *apply_ms,
                                        uint64_t *applies) {
    if (!b) return invalid("NULL batch");
    return read_prof(*b->ws, b->stream, call_ms, calls, apply_ms, applies);
}

// ---------------------------------------------------------------- batches ---
dbtsdf_status dbtsdf_batch_create(void *hip_stream, int use_graph, dbtsdf_batch **out) {
    if (!out) return invalid("NULL out");
    auto b = std::make_unique<dbtsdf_batch>();
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) return check_hip(e, "hipGetDevice");
    b->stream = (hipStream_t)hip_stream;
    if (!b->stream) {
        e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return check_hip(e, "creating the batch stream");
        b->owns_stream = true;
    }
    b->use_graph = use_graph != 0;
    e = hipEventCreateWithFlags(&b->ev, hipEventDisableTiming);
    if (e != hipSuccess) return check_hip(e, "hipEventCreate");
    b->ws = std::make_unique<Workspace>();
    b->ws->device = b->device;
    *out = b.release();
    return DBTSDF_OK;
}

static dbtsdf_status batch_impl(dbtsdf_batch *b, uint32_t n_scans, dbtsdf_grid *const *grids, const float *poses,
                                const float *poses_end, int mode, const float *const *points,
                                const float *const *times, const uint64_t *n, int points_on_device,
                                dbtsdf_scan_stats *stats) {
    TraceRange trace_range("dbtsdf_batch_integrate");
    if (!b) return invalid("NULL batch");
    if (n_scans == 0) return DBTSDF_OK;
    if (!grids || !poses || !points || !n) return invalid("NULL argument");
    if (poses_end && !times) return invalid("NULL times");
    std::vector<float> sweep(poses_end ? 7 * (size_t)n_scans : 0);
    uint64_t total = 0;
    for (uint32_t i = 0; i < n_scans; ++i) {
        if (!grids[i]) return invalid("NULL grid");
        if (grids[i]->device != b->device) return invalid("grid on another device than the batch");
        if (grids[i]->poisoned) return DBTSDF_ERR_POISONED;
        if (n[i] && !points[i]) return invalid("NULL points");
        if (poses_end && n[i] && !times[i]) return invalid("NULL times");
        for (int k = 0; k < 16; ++k)
            if (!std::isfinite(poses[16 * (size_t)i + k])) return invalid("pose must be finite");
        if (poses_end && !sweep_constants(poses + 16 * (size_t)i, poses_end + 16 * (size_t)i, mode, &sweep[7 * i]))
            return invalid("non-finite end pose or unknown deskew mode");
        total += n[i];
    }
    if (total > kMaxPointsPerCall) {
        set_error("too many points in one call");
        return DBTSDF_ERR_OUT_OF_RANGE;
    }
    std::vector<ScanIn> v(n_scans);
    float *stage = nullptr;
    if (!points_on_device) {
        // every scan's points, then (sweeps) every scan's time fractions
        const uint64_t floats = (poses_end ? 4 : 3) * std::max<uint64_t>(total, 1);
        hipError_t e = b->ws->ensure_staging(floats, b->stream);
        if (e != hipSuccess) return check_hip(e, "allocating point staging");
        stage = b->ws->staging;
    }
    // order after earlier work on each grid's own stream
    std::vector<dbtsdf_grid *> distinct;
    for (uint32_t i = 0; i < n_scans; ++i)
        if (std::find(distinct.begin(), distinct.end(), grids[i]) == distinct.end()) distinct.push_back(grids[i]);
    for (dbtsdf_grid *g : distinct) {
        if (g->stream == b->stream || g->external_order) continue;
        hipError_t e = hipEventRecord(g->ev, g->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, g->ev, 0);
        if (e != hipSuccess) return check_hip(e, "ordering the batch after grid work", g);
    }
    uint64_t off = 0;
    for (uint32_t i = 0; i < n_scans; ++i) {
        const float *dev = points[i];
        const float *dev_t = poses_end ? times[i] : nullptr;
        if (!points_on_device && n[i]) {
            hipError_t e = hipMemcpyAsync(stage + 3 * off, points[i], 12 * n[i], hipMemcpyHostToDevice, b->stream);
            if (e == hipSuccess && poses_end)
                e = hipMemcpyAsync(stage + 3 * total + off, times[i], 4 * n[i], hipMemcpyHostToDevice, b->stream);
            if (e != hipSuccess) return check_hip(e, "staging host points");
            dev = stage + 3 * off;
            dev_t = poses_end ? stage + 3 * total + off : nullptr;
        }
        v[i] = ScanIn{grids[i], poses + 16 * (size_t)i, dev, n[i], stats ? &stats[i] : nullptr};
        if (poses_end) {
            v[i].times = dev_t;
            for (int k = 0; k < 4; ++k) v[i].dq[k] = sweep[7 * i + k];
            for (int k = 0; k < 3; ++k) v[i].dt[k] = sweep[7 * i + 4 + k];
        }
        off += n[i];
    }
    dbtsdf_status s = enqueue_scans(*b->ws, b->stream, v, b->use_graph, false);
    if (s != DBTSDF_OK) return s;
    hipError_t e = hipEventRecord(b->ev, b->stream);
    for (dbtsdf_grid *g : distinct)
        if (e == hipSuccess && g->stream != b->stream && !g->external_order) e = hipStreamWaitEvent(g->stream, b->ev, 0);
    return check_hip(e, "ordering grid work after the batch");
}

dbtsdf_status dbtsdf_batch_integrate(dbtsdf_batch *b, uint32_t n_scans, dbtsdf_grid *const *grids, const float *poses,
                                     const float *const *points, const uint64_t *n, int points_on_device,
                                     dbtsdf_scan_stats *stats) {
    return batch_impl(b, n_scans, grids, poses, nullptr, 0, points, nullptr, n, points_on_device, stats);
}

// One batch context per device for dbtsdf_integrate_batch, made on first use
// and kept until the process ends; calls through it are serialised.
dbtsdf_status dbtsdf_integrate_batch(uint32_t n_scans, dbtsdf_grid *const *grids, const float *poses,
                                     const float *const *points, const uint64_t *n, dbtsdf_scan_stats *stats) {
    if (n_scans == 0) return DBTSDF_OK;
    if (!grids || !grids[0]) return invalid("NULL argument");
    static std::mutex mu;
    static std::map<int, dbtsdf_batch *> contexts;
    std::lock_guard<std::mutex> lk(mu);
    dbtsdf_batch *&b = contexts[grids[0]->device];
    if (!b) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess) e = hipSetDevice(grids[0]->device);
        if (e != hipSuccess) return check_hip(e, "selecting the grids' device");
        dbtsdf_status cs = dbtsdf_batch_create(nullptr, 1, &b);
        (void)hipSetDevice(cur);
        if (cs != DBTSDF_OK) {
            b = nullptr;
            return cs;
        }
    }
    dbtsdf_status s = batch_impl(b, n_scans, grids, poses, nullptr, 0, points, nullptr, n, 1, stats);
    // the statistics are delivered by the context's sync, which the caller cannot reach
    if (s == DBTSDF_OK && stats) s = dbtsdf_batch_sync(b);
    return s;
}

dbtsdf_status dbtsdf_batch_integrate_deskew(dbtsdf_batch *b, uint32_t n_scans, dbtsdf_grid *const *grids,
                                            const float *poses_start, const float *poses_end, int mode,
                                            const float *const *points, const float *const *times, const uint64_t *n,
                                            int points_on_device, dbtsdf_scan_stats *stats) {
    if (!poses_end) return invalid("NULL argument");
    return batch_impl(b, n_scans, grids, poses_start, poses_end, mode, points, times, n, points_on_device, stats);
}

dbtsdf_status dbtsdf_batch_sync(dbtsdf_batch *b) {
    if (!b) return invalid("NULL batch");
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return check_hip(e, "synchronising the batch stream");
    b->ws->deliver_all();
    return DBTSDF_OK;
}

dbtsdf_status dbtsdf_batch_graph_stats(const dbtsdf_batch *b, uint64_t *captures, uint64_t *replays) {
    if (!b) return invalid("NULL batch");
    if (captures) *captures = b->ws->captures;
    if (replays) *replays = b->ws->replays;
    return DBTSDF_OK;
}

void dbtsdf_batch_destroy(dbtsdf_batch *b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    b->ws.reset();
    if (b->ev) (void)hipEventDestroy(b->ev);
    if (b->owns_stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // extern "C"

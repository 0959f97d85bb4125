// Autotuner: times candidate launch tunings (brick shape, workgroup size,
// conflict strategy) on a scratch copy of a grid, checks that every candidate
// produces a bit-identical grid, and keeps the fastest.
#include <algorithm>
#include <cstring>
#include <vector>

#include "runtime.h"

using namespace dbtsdf;

namespace {

struct Scratch {
    uint32_t *mask = nullptr, *packed = nullptr, *ref_mask = nullptr, *ref_packed = nullptr;
    unsigned long long *diff = nullptr;
    ~Scratch() {
        void *p[] = {mask, packed, ref_mask, ref_packed, diff};
        for (void *x : p)
            if (x) (void)hipFree(x);
    }
};

std::vector<Tuning> candidates(int K) {
    static const uint32_t shapes[][4] = {{16, 8, 8, 256},  {32, 8, 8, 256},  {64, 8, 8, 256},  {16, 16, 8, 256},
                                         {32, 16, 8, 256}, {32, 16, 8, 512}, {64, 16, 8, 512}, {32, 16, 16, 512}};
    std::vector<Tuning> out;
    for (auto &s : shapes) {
        Tuning t;
        t.strategy = DBTSDF_STRATEGY_BRICK;
        t.bx = s[0];
        t.by = s[1];
        t.bz = s[2];
        t.threads = s[3];
        if (tuning_supported(t, K)) out.push_back(t);
    }
    Tuning a;
    a.strategy = DBTSDF_STRATEGY_ATOMIC;
    a.threads = 256;
    out.push_back(a);
    Tuning tl;
    tl.strategy = DBTSDF_STRATEGY_TILE;
    tl.bx = kTileX;
    tl.by = kTileY;
    tl.bz = kTileZ;
    tl.threads = 256;
    if (tuning_supported(tl, K)) out.push_back(tl);
    Tuning srt;
    srt.strategy = DBTSDF_STRATEGY_SORT;
    srt.threads = 256;
    srt.chunk = 0;
    out.push_back(srt);
    return out;
}

}  // namespace

extern "C" dbtsdf_status dbtsdf_autotune(dbtsdf_grid *g, uint32_t n_scans, const float *poses,
                                         const float *const *points_dev, const uint64_t *n, dbtsdf_tuning *best) {
    if (!g || (n_scans && (!poses || !points_dev || !n))) {
        set_error("NULL argument");
        return DBTSDF_ERR_INVALID_ARG;
    }
    if (g->poisoned) return DBTSDF_ERR_POISONED;
    if (n_scans == 0) return best ? dbtsdf_get_tuning(g, best) : DBTSDF_OK;
    hipStream_t st = g->stream;
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(e, "autotune: synchronising", g);
    const size_t bytes = g->n_voxels * 4;
    Scratch s;
    for (void **p : {(void **)&s.mask, (void **)&s.packed, (void **)&s.ref_mask, (void **)&s.ref_packed}) {
        e = hipMalloc(p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_error("autotune: no room for scratch copies of the grid");
            return DBTSDF_ERR_OUT_OF_MEMORY;
        }
    }
    e = hipMalloc((void **)&s.diff, 8);
    if (e != hipSuccess) return check_hip(e, "autotune: allocation", g);

    // a scratch grid on the scratch planes, same parameters
    dbtsdf_kernel_set ks;
    std::string err;
    ks.ks.reset(build_kernel_set(g->kparams, &err));
    if (!ks.ks) {
        set_error(err);
        return DBTSDF_ERR_INVALID_ARG;
    }
    dbtsdf_grid *tmp = nullptr;
    dbtsdf_status rs = dbtsdf_create_grid_on(&g->params, &ks, st, s.mask, s.packed, &tmp);
    if (rs != DBTSDF_OK) return rs;

    hipEvent_t t0, t1;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    const std::vector<Tuning> cand = candidates(g->K);
    float best_ms = 1e30f;
    Tuning best_t = g->tuning;
    bool have_ref = false;
    dbtsdf_status result = DBTSDF_OK;
    for (const Tuning &c : cand) {
        dbtsdf_tuning ct{};
        ct.strategy = c.strategy;
        ct.brick[0] = c.bx ? c.bx : g->tuning.bx;
        ct.brick[1] = c.by ? c.by : g->tuning.by;
        ct.brick[2] = c.bz ? c.bz : g->tuning.bz;
        ct.block_threads = c.threads;
        ct.apply_blocks = 0;
        ct.chunk = c.chunk ? c.chunk : 0xFFFFFFFFu;
        if (dbtsdf_set_tuning(tmp, &ct) != DBTSDF_OK) continue;
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && result == DBTSDF_OK; ++rep) {  // rep 0 warms up allocations
            e = hipMemcpyAsync(s.mask, g->mask, bytes, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipMemcpyAsync(s.packed, g->packed, bytes, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipEventRecord(t0, st);
            for (uint32_t i = 0; i < n_scans && e == hipSuccess; ++i) {
                rs = dbtsdf_integrate_scan(tmp, poses + 16 * (size_t)i, points_dev[i], n[i], 1, nullptr);
                if (rs != DBTSDF_OK) result = rs;
            }
            if (e == hipSuccess) e = hipEventRecord(t1, st);
            if (e == hipSuccess) e = hipEventSynchronize(t1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
            if (e != hipSuccess) result = check_hip(e, "autotune: timing", g);
        }
        if (result != DBTSDF_OK) break;
        if (!have_ref) {
            e = hipMemcpyAsync(s.ref_mask, s.mask, bytes, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipMemcpyAsync(s.ref_packed, s.packed, bytes, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) {
                result = check_hip(e, "autotune: reference copy", g);
                break;
            }
            have_ref = true;
        } else {
            unsigned long long diff = 0;
            e = hipMemsetAsync(s.diff, 0, 8, st);
            if (e == hipSuccess) e = launch_count_diff(s.mask, s.ref_mask, g->n_voxels, s.diff, st);
            if (e == hipSuccess) e = launch_count_diff(s.packed, s.ref_packed, g->n_voxels, s.diff, st);
            if (e == hipSuccess) e = hipMemcpyAsync(&diff, s.diff, 8, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) {
                result = check_hip(e, "autotune: compare", g);
                break;
            }
            if (diff != 0) {
                set_error("autotune: a candidate tuning produced a different grid");
                result = DBTSDF_ERR_DEVICE;
                break;
            }
        }
        if (ms < best_ms) {
            best_ms = ms;
            best_t = tmp->tuning;
            best_t.apply_blocks = 0;
        }
    }
    dbtsdf_destroy_grid(tmp);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (result != DBTSDF_OK) return result;
    dbtsdf_tuning bt{};
    bt.strategy = best_t.strategy;
    bt.brick[0] = best_t.bx;
    bt.brick[1] = best_t.by;
    bt.brick[2] = best_t.bz;
    bt.block_threads = best_t.threads;
    bt.apply_blocks = 0;
    bt.chunk = best_t.chunk ? best_t.chunk : 0xFFFFFFFFu;
    rs = dbtsdf_set_tuning(g, &bt);
    if (rs != DBTSDF_OK) return rs;
    if (best) *best = bt;
    return DBTSDF_OK;
}

// Host runtime objects behind the C ABI: grids, workspaces, batch contexts.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <memory>
#include <string>
#include <vector>

#include "internal.h"

namespace dbtsdf {
struct DeviceTables;
}

struct dbtsdf_kernel_set {
    std::unique_ptr<dbtsdf::KernelSet> ks;
    // device copies of the tables, one per device, shared by the grids made
    // from this kernel set (and kept alive by them)
    std::mutex mu;
    std::map<int, std::shared_ptr<dbtsdf::DeviceTables>> dev;
};

namespace dbtsdf {

void set_error(const std::string &msg);

// Device copy of one kernel set.
struct DeviceTables {
    DevTables t{};
    std::vector<void *> allocs;
    dbtsdf_kernel_params params{};
    uint32_t max_shadow = 0;   // cells of the largest shadow set
    ~DeviceTables();
};

// One call's statistics waiting for delivery.
struct PendingStat {
    dbtsdf_scan_stats *dst;
    uint32_t scan;           // index into the call's scan counters
    int32_t traffic_grid;    // grid whose traffic counters go on this scan, or -1
    uint64_t n_in;
    uint64_t k3;
};

struct RingSlot {
    void *host = nullptr;    // pinned, coherent: descriptors, then the counters written back
    void *host_dev = nullptr;  // the same buffer's device address
    size_t bytes = 0;
    hipEvent_t ev = nullptr;
    bool busy = false;
    size_t ctr_off = 0;      // byte offset of the counters inside host
    std::vector<PendingStat> pend;
    hipEvent_t pe[3] = {nullptr, nullptr, nullptr};  // call start, apply start, apply/call end
    int prof = 0;            // 0: none, 1: whole call, 2: call and apply kernel
};

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
};

// Buffers of the sort strategy (allocated on its first call, grown as calls
// need): pairs twice over for the radix sort, the pair counter and the sort's
// temporary storage.
struct SortBuffers {
    unsigned long long *keys[2] = {nullptr, nullptr};
    uint32_t *vals[2] = {nullptr, nullptr};
    size_t cap = 0;               // pairs each buffer holds
    uint32_t *cnt = nullptr, *off = nullptr;
    size_t surv_cap = 0;          // entries of cnt and off
    unsigned long long *bits = nullptr;
    size_t bits_cap = 0;          // ballot words
    void *tmp = nullptr;          // the scan's and the sort's temporary storage
    size_t tmp_bytes = 0;
};
// The key layout and launch shape of one sort-strategy call.
struct SortPlan {
    uint32_t shift;               // voxel-index bits of a key (grid index above them)
    uint32_t end_bit;             // key bits in use
    uint32_t emit_blocks;
    unsigned long long pairs_per_point;  // most pairs one return emits: K^3 + largest shadow set
    uint32_t round_survivors;     // most survivors per round (0: as many as the buffers allow)
    uint32_t words;               // ballot words per survivor: window passes + shadow passes
};

// Stream-ordered scratch for integrate calls (one per grid for the plain
// entry point, one per batch context).
struct Workspace {
    int device = 0;
    uint32_t points_cap = 0, scans_cap = 0, grids_cap = 0, items_cap = 0, entries_cap = 0;
    uint32_t hash_cap = 0;
    void *d_desc = nullptr;          // Ctrl | CallInfo | DevGrid[grids_cap] | DevScan[scans_cap]
    size_t desc_bytes = 0;
    uint4 *rec = nullptr;
    uint32_t *pslot = nullptr;
    unsigned long long *hkeys = nullptr;
    uint32_t *hvals = nullptr;
    unsigned long long *items = nullptr;
    uint32_t *item_off = nullptr, *item_cnt = nullptr;
    uint4 *entries = nullptr;
    uint32_t *rank = nullptr;
    uint4 *work = nullptr;
    unsigned long long *ctr = nullptr;   // scan counters then traffic counters
    float *staging = nullptr;            // device copy of host points
    size_t staging_cap = 0;              // floats
    std::vector<RingSlot> ring;
    uint32_t ring_next = 0;
    std::map<std::string, GraphEntry> graphs;
    hipStream_t cap_stream = nullptr;    // private stream the graphs are captured on
    uint64_t captures = 0, replays = 0;
    uint32_t prof_every = 0;             // time every prof_every-th call (0: profiling off)
    uint64_t n_calls = 0;                // integrate calls enqueued on this workspace
    SortBuffers sorter;
    double prof_call_ms = 0.0, prof_apply_ms = 0.0;
    uint64_t prof_calls = 0, prof_apply = 0;

    ~Workspace();
    hipError_t ensure(uint32_t n_points, uint32_t n_scans, uint32_t n_grids, uint32_t entry_factor,
                      hipStream_t st);
    hipError_t ensure_staging(size_t floats, hipStream_t st);
    RingSlot &next_slot(size_t bytes, std::string *err);
    void deliver(RingSlot &s);
    void deliver_all();
    void drop_graphs();
    void release();
};

void free_sort_buffers(SortBuffers &b);
// The sort strategy's apply (sort_reduce.hip): reads the survivor count back,
// then per round of survivors emits, sorts and reduces the pairs on stream st.
hipError_t sort_apply(Workspace &ws, const PipeArgs &a, const SortPlan &plan, hipStream_t st);

}  // namespace dbtsdf

struct dbtsdf_grid {
    dbtsdf_grid_params params{};
    dbtsdf_kernel_params kparams{};
    int K = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    bool owns_planes = true;
    uint32_t *mask = nullptr;
    uint32_t *packed = nullptr;
    uint64_t n_voxels = 0;
    std::shared_ptr<dbtsdf::DeviceTables> tables;
    dbtsdf::Tuning tuning;
    uint32_t *brick_cnt = nullptr;
    uint32_t *brick_slot = nullptr;
    uint32_t nb[3] = {0, 0, 0};
    uint32_t brick_dims[3] = {0, 0, 0};
    std::unique_ptr<dbtsdf::Workspace> ws;
    hipEvent_t ev = nullptr;
    // the planes were changed only by integration since creation or the last
    // reset (a return in a voxel integrated by an earlier call can then skip
    // its eq. 4 window); dbtsdf_write_voxels clears it
    bool revisit_skip = true;
    // mesh export: the case table on the device and the triangle counter
    uint32_t *mesh_table = nullptr;
    unsigned long long *mesh_count = nullptr;
    bool poisoned = false;
    // set by the server, which orders all work on its grids itself: batches
    // then skip the event handshake with the grid's own stream
    bool external_order = false;
};

struct dbtsdf_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    bool use_graph = true;
    std::unique_ptr<dbtsdf::Workspace> ws;
    hipEvent_t ev = nullptr;
    std::vector<dbtsdf_grid *> last_grids;
};

namespace dbtsdf {

struct ScanIn {
    dbtsdf_grid *grid;
    const float *pose;     // 16 floats, host
    const float *points;   // device pointer (after staging)
    uint64_t n;            // points taken
    dbtsdf_scan_stats *stats;
    uint32_t step = 1;     // every step-th point of the array
    // a motion-compensated sweep: per-return time fractions (device) and the
    // sweep's constants (sweep_constants); pose is the start pose
    const float *times = nullptr;
    float dq[4] = {1.0f, 0.0f, 0.0f, 0.0f};
    float dt[3] = {0.0f, 0.0f, 0.0f};
};
// The constants of a sweep (deskew.cpp): q (w, x, y, z) then t1 - t0; false
// for a non-finite pose or an unknown mode.
bool sweep_constants(const float p0[16], const float p1[16], int mode, float out[7]);

// The device descriptors of a grid (index: its place in the call) and of a scan.
DevGrid dev_grid_of(const dbtsdf_grid *g, uint32_t index);
DevScan dev_scan_of(const ScanIn &s, uint32_t begin, uint32_t grid_index);
bool row_kernel_covers(const dbtsdf_grid *g);
bool row_kernel_tables(const dbtsdf_grid *g);

// Validates and enqueues one call (plain or batched) on stream st using ws.
dbtsdf_status enqueue_scans(Workspace &ws, hipStream_t st, std::vector<ScanIn> &scans, bool use_graph, bool plain);
dbtsdf_status ensure_bricks(dbtsdf_grid *g);
dbtsdf_status check_hip(hipError_t e, const char *what, dbtsdf_grid *g = nullptr);

}  // namespace dbtsdf

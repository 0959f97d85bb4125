// The allocation-free variant of the plain one-scan call
// (dbtsdf_integrate_scan_noalloc): the same per-point passes (front end with
// first-return dedup, survivor selection, apply) as dbtsdf_integrate_scan
// with the per-point strategy, with every buffer the call needs beyond the
// grid and the caller's points held in one static device array per GPU.
//
// The array's name in host code is a host-side stand-in, not a device
// address: its device address is taken once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// passed to kernels and copies.
#include <cmath>
#include <cstring>
#include <mutex>

#include "runtime.h"

namespace dbtsdf {

// Largest scan one call takes (points), and the dedup table (a power of two
// of at least twice that, so an empty slot always exists and probes stay
// short).
constexpr uint32_t kNoAllocPoints = DBTSDF_NOALLOC_MAX_POINTS;
constexpr uint32_t kNoAllocHash = 4u * kNoAllocPoints;
constexpr uint32_t kNoAllocGrids = 2;   // descriptor slots: the scan descriptor then starts on 16 bytes

// Byte layout of the scratch array.
constexpr size_t kHostDescBytes = sizeof(CallInfo) + kNoAllocGrids * sizeof(DevGrid) + sizeof(DevScan);
constexpr size_t kScansOff = sizeof(CallInfo) + kNoAllocGrids * sizeof(DevGrid);
static_assert(kScansOff % 16 == 0, "the one-scan front pass reads the scan descriptor in 16-byte pieces");
constexpr size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
constexpr size_t kOffHostDesc = 0;                                               // as the host lays it out
constexpr size_t kOffDesc = align256(kOffHostDesc + kHostDescBytes);             // Ctrl | the device copy
constexpr size_t kOffCtr = align256(kOffDesc + sizeof(Ctrl) + kHostDescBytes);   // scan then traffic counters
constexpr size_t kCtrWords = SC_N + kNoAllocGrids * TC_N;
constexpr size_t kOffOut = align256(kOffCtr + kCtrWords * 8);                    // the statistics written out
constexpr size_t kOffRec = align256(kOffOut + kCtrWords * 8);
constexpr size_t kOffPslot = align256(kOffRec + (size_t)kNoAllocPoints * sizeof(uint4));
constexpr size_t kOffKeys = align256(kOffPslot + (size_t)kNoAllocPoints * 4);
constexpr size_t kOffVals = align256(kOffKeys + (size_t)kNoAllocHash * 8);
constexpr size_t kOffSurv = align256(kOffVals + (size_t)kNoAllocHash * 4);
constexpr size_t kScratchBytes = align256(kOffSurv + (size_t)kNoAllocPoints * sizeof(uint4));
static_assert(kScratchBytes == DBTSDF_NOALLOC_SCRATCH_BYTES, "the header states the scratch size");

}  // namespace dbtsdf

// One copy per GPU the library runs on, held until the process ends.
static __device__ __align__(256) unsigned char scratch[dbtsdf::kScratchBytes];

namespace dbtsdf {

namespace {

struct NoAllocDevice {
    std::once_flag once;
    hipError_t init_err = hipSuccess;
    unsigned char *ptr = nullptr;   // device address of this device's scratch array
    int apply_blocks_row = 0, apply_blocks_generic = 0;
};

constexpr int kMaxDevices = 64;
NoAllocDevice g_dev[kMaxDevices];

// Set-up on the first call on a device (that device current): the array's
// device address, the dedup table emptied, the apply grids sized.
void init_device(NoAllocDevice &d, int device, hipStream_t st) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        d.init_err = e;
        return;
    }
    unsigned char *base = static_cast<unsigned char *>(p);
    e = launch_fill_u64(reinterpret_cast<unsigned long long *>(base + kOffKeys), kHashEmpty, kNoAllocHash, st);
    if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<uint32_t *>(base + kOffVals), 0xFFFFFFFFu, kNoAllocHash, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        d.init_err = e;
        return;
    }
    Tuning t;
    t.strategy = DBTSDF_STRATEGY_ATOMIC;
    d.apply_blocks_row = apply_blocks_default(t, 11, true, device);
    d.apply_blocks_generic = apply_blocks_default(t, kMaxK, false, device);
    d.ptr = base;
}

}  // namespace
}  // namespace dbtsdf

using namespace dbtsdf;

extern "C" dbtsdf_status dbtsdf_integrate_scan_noalloc(dbtsdf_grid *g, const float pose[16], const float *points_dev,
                                                       uint64_t n, dbtsdf_scan_stats *stats) {
    if (!g || !pose) {
        set_error("NULL argument");
        return DBTSDF_ERR_INVALID_ARG;
    }
    if (g->poisoned) {
        set_error("grid is poisoned by an earlier device error");
        return DBTSDF_ERR_POISONED;
    }
    for (int k = 0; k < 16; ++k)
        if (!std::isfinite(pose[k])) {
            set_error("pose must be finite");
            return DBTSDF_ERR_INVALID_ARG;
        }
    if (n > kNoAllocPoints) {
        set_error("dbtsdf_integrate_scan_noalloc takes at most DBTSDF_NOALLOC_MAX_POINTS points per call");
        return DBTSDF_ERR_OUT_OF_RANGE;
    }
    if (n && !points_dev) {
        set_error("NULL points");
        return DBTSDF_ERR_INVALID_ARG;
    }
    if (n == 0) {
        if (stats) *stats = dbtsdf_scan_stats{};
        return DBTSDF_OK;
    }
    if (g->device < 0 || g->device >= kMaxDevices) {
        set_error("device index out of range");
        return DBTSDF_ERR_INVALID_ARG;
    }
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != g->device) e = hipSetDevice(g->device);
    if (e != hipSuccess) return check_hip(e, "selecting the grid's device", g);
    NoAllocDevice &dev = g_dev[g->device];
    std::call_once(dev.once, init_device, std::ref(dev), g->device, g->stream);
    if (dev.init_err != hipSuccess || !dev.ptr) {
        if (cur != g->device) (void)hipSetDevice(cur);
        return check_hip(dev.init_err != hipSuccess ? dev.init_err : hipErrorInvalidValue,
                         "setting up the allocation-free scratch", g);
    }
    unsigned char *base = dev.ptr;

    // descriptors, laid out as on the host ring of the plain call: CallInfo |
    // DevGrid[2] | DevScan
    alignas(16) unsigned char desc[kHostDescBytes] = {};
    const CallInfo ci{(uint32_t)n, 1u, 1u, 0u};
    std::memcpy(desc, &ci, sizeof(ci));
    const DevGrid dg = dev_grid_of(g, 0u);
    std::memcpy(desc + sizeof(CallInfo), &dg, sizeof(dg));
    ScanIn in{g, pose, points_dev, n, nullptr, 1u};
    const DevScan ds = dev_scan_of(in, 0u, 0u);
    std::memcpy(desc + kScansOff, &ds, sizeof(ds));
    e = hipMemcpyAsync(base + kOffHostDesc, desc, kHostDescBytes, hipMemcpyHostToDevice, g->stream);

    const bool row = row_kernel_covers(g);
    Tuning tun;
    tun.strategy = DBTSDF_STRATEGY_ATOMIC;
    tun.apply_blocks = (uint32_t)(row ? dev.apply_blocks_row : dev.apply_blocks_generic);
    PipeArgs a{};
    a.ctrl = reinterpret_cast<Ctrl *>(base + kOffDesc);
    a.grids = reinterpret_cast<const DevGrid *>(base + kOffDesc + sizeof(Ctrl) + sizeof(CallInfo));
    a.scans = reinterpret_cast<const DevScan *>(base + kOffDesc + sizeof(Ctrl) + kScansOff);
    a.tab = g->tables->t;
    a.hash_mask = kNoAllocHash - 1u;
    a.rec = reinterpret_cast<uint4 *>(base + kOffRec);
    a.pslot = reinterpret_cast<uint32_t *>(base + kOffPslot);
    a.hkeys = reinterpret_cast<unsigned long long *>(base + kOffKeys);
    a.hvals = reinterpret_cast<uint32_t *>(base + kOffVals);
    a.surv_rec = reinterpret_cast<uint4 *>(base + kOffSurv);
    a.entries = a.surv_rec;
    a.scan_ctr = reinterpret_cast<unsigned long long *>(base + kOffCtr);
    a.traffic_ctr = a.scan_ctr + SC_N;
    a.host_desc = reinterpret_cast<const uint2 *>(base + kOffHostDesc);
    a.host_ctr = reinterpret_cast<unsigned long long *>(base + kOffOut);
    a.desc_scans_off = (uint32_t)kScansOff;
    a.scans_cap = 1u;
    a.single_scan = 1u;
    a.row_kernel = row ? 1u : 0u;
    a.revisit_ok = g->tables->t.n_bins <= 32768u ? 1u : 0u;
    if (e == hipSuccess) e = launch_pipeline(a, tun, kNoAllocPoints, g->stream, kPartAll);
    if (e != hipSuccess) {
        if (cur != g->device) (void)hipSetDevice(cur);
        return check_hip(e, "launching the integration kernels", g);
    }
    if (stats) {
        unsigned long long c[kCtrWords] = {};
        e = hipMemcpyAsync(c, base + kOffOut, sizeof(c), hipMemcpyDeviceToHost, g->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) {
            if (cur != g->device) (void)hipSetDevice(cur);
            return check_hip(e, "reading the statistics back", g);
        }
        dbtsdf_scan_stats st{};
        const uint64_t k3 = (uint64_t)g->K * g->K * g->K;
        st.n_in = n;
        st.n_invalid = c[SC_INVALID];
        st.n_out_of_bounds = c[SC_OOB];
        st.n_duplicate = c[SC_DUP];
        st.n_integrated = c[SC_INT];
        st.voxel_updates = c[SC_INT] * k3;
        st.shadow_updates = c[SC_SHADOW];
        st.n_revisit = c[SC_REVISIT];
        *stats = st;
    }
    if (cur != g->device) (void)hipSetDevice(cur);
    return DBTSDF_OK;
}

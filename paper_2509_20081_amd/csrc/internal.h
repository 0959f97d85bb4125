// Internal types shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/dbtsdf.h"

namespace dbtsdf {

// ---------------------------------------------------------------- limits ---
constexpr int kMaxK = 37;                       // eq. 3 masks stay within 32 bits
constexpr uint32_t kMaxDim = 1u << 20;          // per axis
constexpr uint64_t kMaxPointsPerCall = 1ull << 28;
constexpr uint64_t kMaxScansPerCall = 1ull << 20;
constexpr int kVoxelKeyBits = 40;               // dedup key = scan << 40 | linear voxel
constexpr uint64_t kHashEmpty = ~0ull;
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
constexpr uint32_t kMaxAtomicGrids = 1u << 16;  // per-point strategy: grid index in 16 bits of a survivor record

// point record word w: bits 0-15 direction bin, bits 16-17 status,
// bit 30 set by the select pass on returns that are integrated
constexpr uint32_t kStOk = 0, kStInvalid = 1, kStOob = 2;
constexpr uint32_t kRecSurvivor = 1u << 30;
// survivor record word (per-point and sort strategies): bin in bits 0-15
// (bits 0-14 and the revisit flag in bit 15 when the kernel set has at most
// 32768 bins, PipeArgs::revisit_ok), grid index in bits 16-31
constexpr uint32_t kRecRevisit = 1u << 15;
constexpr uint32_t kRowBinMask = kRecRevisit - 1u;
// point record word, tile strategy: the front pass found the return's voxel
// integrated by an earlier call (its window is skipped)
constexpr uint32_t kRecTileRevisit = 1u << 29;
// tile strategy: list entries of returns that lost the first-return test
constexpr uint32_t kTileHole = 0xFFFFFFFFu;
// The tile strategy's grid tiles (x fastest): 128-byte rows of words, 4096
// words a tile.
constexpr uint32_t kTileX = 32, kTileY = 16, kTileZ = 8;

// ------------------------------------------------------- host kernel set ---
struct KernelSet {
    dbtsdf_kernel_params p{};
    int K = 0, R = 0;
    uint32_t n_bins = 0;
    std::vector<uint32_t> cell_mask;     // K^3, index ((dz+R)*K + (dy+R))*K + (dx+R)
    std::vector<uint32_t> mask_by_q;     // mask by metric value q (L2: q = |o|^2, L1: q = |o|_1)
    std::vector<uint8_t> shadow;         // n_bins * K^3 flags
    std::vector<double> dirs;            // n_bins * 3
    std::vector<uint32_t> sh_start;      // n_bins + 1 (CSR of shadow offsets)
    std::vector<uint32_t> sh_off;        // packed (dx+R) | (dy+R) << 8 | (dz+R) << 16
    // AZEL boundary tables (fp32, index k = 1..B_az/2-1 and 1..B_el-1, slot 0 unused)
    std::vector<float> az_c, az_s, el_s2;
    std::vector<uint32_t> el_neg;
    std::vector<uint32_t> row_image;     // kImgWords, or empty when the row kernel does not cover the set
};

KernelSet *build_kernel_set(const dbtsdf_kernel_params &p, std::string *err);

// The LDS tables of the per-point row kernel, laid out as the kernel holds
// them and copied in whole by every workgroup (16-byte words):
//   mtab[sel][row]   sel = 4 qd - a + 3 (lane quad qd, window phase a), row =
//                    (dy + R) + K (dz + R): the eq. 3 masks of cells dx = sel -
//                    3 - R + j, j = 0..3, as int16 pairs (-1 outside the window)
//   sh_pk[j]         the shadow cells of every bin, (dx+R) | (dy+R) << 8 | (dz+R) << 16
//   sh_bits[b][w]    bin b's shadow set as bits (dx+3) + 7 (dy+3) + 49 (dz+3)
//   sh_rng[b]        start of bin b's cells in sh_pk, and the end after the last bin
// Built only for kernel sets the row kernel covers: K <= 11, at most 31 bins,
// r_s^2 <= 9 (cells in [-3, 3]^3, at most 128 per bin, 2048 in all) and masks
// below 2^15.
constexpr uint32_t kRowPad = 128;          // >= K^2 for K <= 11
constexpr uint32_t kRowSel = 16;
constexpr uint32_t kShadowTable = 2048;
constexpr uint32_t kShadowSetWords = 11;   // 7^3 = 343 bits
constexpr uint32_t kRowBins = 32;          // sh_rng entries: at most 31 bins and the end
constexpr uint32_t kImgMtab = 0, kImgShPk = kRowSel * kRowPad * 2, kImgShBits = kImgShPk + kShadowTable,
                   kImgShRng = kImgShBits + kRowBins * kShadowSetWords,
                   kImgWords = (kImgShRng + kRowBins + 1023) / 1024 * 1024;  // whole rounds of 256 16-byte copies
static_assert(kImgWords % 4 == 0 && kImgShPk % 4 == 0 && kImgShBits % 4 == 0 && kImgShRng % 4 == 0,
              "16-byte sections");
bool build_row_image(const KernelSet &ks, std::vector<uint32_t> &img);
int host_bin(const KernelSet &ks, float dx, float dy, float dz);

// ---------------------------------------------------- device descriptors ---
// Kernel tables as the device reads them (one copy per grid).
struct DevTables {
    const uint32_t *mask_by_q;   // n_q entries
    const uint32_t *sh_start;    // n_bins + 1
    const uint32_t *sh_off;      // total shadow cells
    const float *az_c, *az_s, *el_s2;
    const uint32_t *el_neg;
    const uint4 *row_image;  // the row kernel's LDS tables, or null
    uint32_t n_q;
    uint32_t n_bins;
    int32_t K, R;
    int32_t shadow_r2;       // r_s^2, negative = no shadow
    uint32_t binning, bins_az, bins_el, metric;
    uint32_t shadow_model;   // dbtsdf_shadow_model
};

struct DevGrid {
    uint32_t *mask;
    uint32_t *packed;
    uint32_t *brick_cnt;   // per brick: entries this call (reset by the apply pass)
    uint32_t *brick_slot;  // per brick: work-item index this call
    uint32_t nx, ny, nz;
    uint32_t nbx, nby, nbz;
    uint32_t T, hmax;
    uint32_t traffic_slot; // index into traffic counters
    uint32_t revisit_skip; // the planes hold only what integration wrote (see k_select_atomic)
};

struct DevScan {
    float rot[9];          // pose rows 0..2, columns 0..2
    float trans[3];
    float origin[3];
    float inv_s;           // fl32(1 / voxel_size)
    const float *pts;      // the scan's points: point j is pts[3 j step .. 3 j step + 2], fp32, device
    uint32_t begin;        // offset of the scan's first point in the call
    uint32_t n;            // points taken (every step-th of the array)
    uint32_t grid;         // index into DevGrid array
    uint32_t dedup;
    uint32_t step;         // sequential downsampling: every step-th return of the array
    uint32_t deskew;       // 1: a motion-compensated sweep (the fields below)
    float dq[4];           // quaternion (w, x, y, z) of the rotation over the sweep, fp32
    float dt[3];           // end translation - start translation (rot, trans: the start pose)
    float pad1;
    const float *times;    // per return of the array: time fraction in [0, 1], device
    uint32_t pad2[2];
};
static_assert(sizeof(DevScan) % 16 == 0, "DevScan is read in 16-byte pieces");

// Per-scan counters (u64) and per-grid traffic counters.
enum { SC_INVALID = 0, SC_OOB, SC_DUP, SC_INT, SC_SHADOW, SC_REVISIT, SC_N };
enum { TC_UMASK = 0, TC_CMASK, TC_USHADOW, TC_N };

struct Ctrl {
    uint32_t n_active;       // bricks touched this call (work items of the bucketing)
    uint32_t total_entries;  // (point, brick) pairs listed
    uint32_t n_survivors;    // integrated points (atomic strategy)
    uint32_t n_work;         // apply work units (bricks, heavy ones split)
    uint32_t select_done;    // workgroups of the select pass that have finished (atomic strategy)
    uint32_t work_next;      // tile strategy: work items claimed by the apply's workgroups
    uint32_t pad[2];
};

// Sizes of the current call, read by the kernels from device memory so that a
// captured graph can be replayed for any call that fits its capacity.
struct CallInfo {
    uint32_t n_points, n_scans, n_grids, pad;
};

// Everything the pipeline kernels read. Pointers into one workspace.
struct PipeArgs {
    const DevScan *scans;
    const DevGrid *grids;
    DevTables tab;
    uint32_t brick[3];
    uint32_t hash_mask;      // capacity - 1
    uint4 *rec;              // per point: voxel x, y, z and the record word w
    uint32_t *pslot;         // per point hash slot
    unsigned long long *hkeys;
    uint32_t *hvals;
    unsigned long long *items;  // active (grid << 32 | brick)
    uint32_t *item_off;      // first entry of each active brick
    uint32_t *item_cnt;      // entries of each active brick
    uint4 *entries;          // (voxel x, y, z, bin) of the listed points, grouped by brick
    uint32_t *rank;          // per (point, brick) pair: position in the brick's list
    uint4 *work;             // apply work units: (brick, grid, first entry, count | split << 31)
    uint4 *surv_rec;         // per-point strategy: compacted survivors (voxel x, y, z, bin | grid << 16)
    unsigned long long *scan_ctr;     // n_scans * SC_N
    unsigned long long *traffic_ctr;  // n_grids * TC_N
    Ctrl *ctrl;              // followed in memory by the CallInfo
    uint32_t items_cap;
    uint32_t entries_cap;
    uint32_t count_traffic;
    uint32_t span[3];        // most bricks a K^3 cube can touch per axis
    uint32_t chunk;          // listed points per apply work unit (0 = never split a brick)
    uint32_t row_kernel;     // the per-point strategy's apply is the row kernel: the kernel set has its
                             // tables and every grid has Nx % 4 == 0 (16-byte aligned rows) and window
                             // byte offsets that fit 32 bits (8 R (1 + Nx + Nx Ny) < 2^32)
    uint32_t single_scan;    // the call holds exactly one scan (one grid)
    uint32_t tile_mode;      // the tile strategy: per-grid counters indexed through tile_ctr, list offsets
                             // beside them
    uint32_t revisit_ok;     // the kernel set has at most 32768 bins: bit 15 of a survivor's record
                             // word is free for the revisit flag (else the bin uses bits 0-15)
    // the call's descriptors are read from, and its counters written to, the
    // pinned host buffer of its ring slot by the first and last passes
    const uint2 *host_desc;  // CallInfo | DevGrid[grids_cap] | DevScan[n_scans]
    unsigned long long *host_ctr;  // scan counters then traffic counters, as ctrl's copy
    uint32_t desc_scans_off; // byte offset of the DevScan array in the descriptors
    uint32_t scans_cap;      // counters layout: scans_cap * SC_N scan counters first
};

// Sort strategy: every change a return makes to a voxel word becomes a pair
// (key = grid << shift | voxel index, contribution). A contribution is an
// eq. 3 mask (2^n - 1 with n <= 31, so bit 31 clear: an all-ones mask changes
// no word and is never emitted) or kHitPair, one shadow hit.
constexpr uint32_t kHitPair = 0xFFFFFFFFu;
constexpr unsigned long long kSortMaxPairs = 1ull << 28;  // pairs of one round
struct SortArgs {
    void *keys;                  // uint32_t keys when they fit 31 bits, else unsigned long long
    uint32_t *vals;
    unsigned long long *bits;    // per survivor of the round: need ballots of its window and shadow passes
    uint32_t *cnt;               // per survivor of the round: pairs it emits
    uint32_t *off;               // their exclusive sum: where its pairs start
    uint32_t shift;              // voxel-index bits of a key
    uint32_t words;              // ballot words per survivor
    uint32_t surv_lo, surv_hi;   // the survivors of this round
};
constexpr int kSortThreads = 256;
const void *sort_emit_kernel();  // for occupancy queries (kSortThreads per workgroup)

// ---------------------------------------------------------- launch config ---
struct Tuning {
    uint32_t strategy = DBTSDF_STRATEGY_ATOMIC;  // the faster form on dense LiDAR scans
    uint32_t bx = 32, by = 8, bz = 8;
    uint32_t threads = 256;
    uint32_t apply_blocks = 0;
    uint32_t chunk = 64;     // listed points per apply work unit, 0 = never split
};

bool tuning_supported(const Tuning &t, int K);

// Kernel launchers (kernels.hip). Return hipSuccess or the first launch error.
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t st);
// the call's statistics into its ring slot (for apply passes that do not write them)
hipError_t launch_stats_out(const PipeArgs &a, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, uint64_t n, hipStream_t st);
hipError_t launch_grid_init(uint32_t *mask, uint32_t *packed, uint64_t n, hipStream_t st);
// The pass sequence of one call: all of it, or the passes before the apply,
// the apply alone, and the passes after it (the split lets profiling bracket
// the apply kernel with events).
enum { kPartAll = 0, kPartPre = 1, kPartApply = 2, kPartPost = 3 };
// The per-point strategy writes the statistics from its select pass: it has
// no passes after the apply.
inline bool per_point_front(const Tuning &t) {
    return t.strategy == DBTSDF_STRATEGY_ATOMIC || t.strategy == DBTSDF_STRATEGY_SORT;
}
// Only the brick strategy has passes after the apply (k_download).
inline bool pipeline_has_post(const Tuning &t) { return t.strategy == DBTSDF_STRATEGY_BRICK; }
hipError_t launch_pipeline(const PipeArgs &a, const Tuning &t, uint32_t points_cap, hipStream_t st, int part);
hipError_t launch_read_distance(const uint32_t *mask, const uint32_t *packed, int8_t *out, uint64_t n,
                                hipStream_t st);
// Copy box [lo, hi) of one plane (x fastest) into out; with packed != null,
// write the int8 signed distance instead (out is then int8_t*).
hipError_t launch_gather_box(const uint32_t *plane, const uint32_t *packed, const uint32_t dims[3],
                             const uint32_t lo[3], const uint32_t hi[3], void *out, hipStream_t st);
// Number of positions where a != b (n words), added into *count.
hipError_t launch_count_diff(const uint32_t *a, const uint32_t *b, uint64_t n, unsigned long long *count,
                             hipStream_t st);
// ------------------------------------------------------------ mesh export ---
// Marching Cubes case table (mesh.cpp): per corner case (bit c set = corner c
// inside), byte 0 the triangle count, byte 1 the loop count, then per loop a
// header (vertex count m | 16 when fanned from its centre) and its m edge
// numbers, from the smallest.
constexpr uint32_t kMeshCaseBytes = 24;
// Per case, the same triangles listed one by one (in the loops' order): three
// vertex codes each, an edge number (0-11), or kMeshCentre | p for the centre
// of the loop whose header sits at byte p of the case's entry in b.
constexpr uint32_t kMeshTriBytes = 24;   // at most 7 triangles per case
constexpr uint8_t kMeshCentre = 0x80;
struct MeshTable {
    uint8_t b[256][kMeshCaseBytes];
    uint8_t tri[256][kMeshTriBytes];
};
const MeshTable &mesh_table();

struct MeshArgs {
    const uint32_t *mask;
    const uint32_t *packed;
    const uint32_t *table;       // the MeshTable on the device
    float *out;                  // 9 floats per triangle, or null (count only)
    unsigned long long *count;   // triangles found (reset by the caller)
    unsigned long long cap;      // triangles out can hold
    uint32_t nx, ny;             // grid dimensions (plane strides)
    uint32_t lo[3];              // first cube (its lower corner voxel)
    uint32_t nc[3];              // cubes per axis
    float origin[3];
    float s;
};
hipError_t launch_mesh(const MeshArgs &m, hipStream_t st);
// Point export: centres of the occupied contact voxels (mask 0, sign 0) of the
// box lo + [0, nc) (MeshArgs.nc holds the box extent here, MeshArgs.table is
// unused), 3 floats each.
hipError_t launch_points(const MeshArgs &m, hipStream_t st);

// Workgroups of a fully resident persistent apply grid (row_kernel: the
// kernel set has the row kernel's tables).
int apply_blocks_default(const Tuning &t, int K, bool row_kernel, int device);

}  // namespace dbtsdf

// gfx950 kernels of DB-TSDF scan integration (Sec. III-C of the paper).
//
// One call integrates a set of scans (one for the plain entry point, many for
// the batched one) through this pass sequence on one stream (launched
// directly, or replayed from a captured graph):
//
//   k_upload   the call's descriptors from its pinned host ring slot
//   k_reset    zero the per-call counters
//   k_front    per point: fp32 transform into the map frame, validity,
//              voxelisation, K^3 bounds test, direction bin (eq. 2); the
//              first-return-per-voxel rule (Sec. IV-B) by an atomicMin of the
//              point index into a hash table keyed by (scan, voxel)
//   then one of two strategies, with identical results:
//   per point (a one-scan call folds k_upload and k_reset into k_front, and
//   k_download into the apply pass: three passes in all)
//     k_select_atomic  survivor test, compacted survivor records, per-scan
//                      statistics, release of the hash slots (the apply
//                      pass's workgroup 0 writes the statistics out)
//     k_apply_points   one wavefront per survivor: the K^3 window in aligned
//                      16-byte rows, eq. 4 by read-first atomicAnd, eqs. 5-6
//                      by guard-bit counter atomics (k_apply_atomic: any K)
//   per brick
//     k_select_pairs   survivor test; bucketing of survivors by the grid
//                      bricks their K^3 cube touches (the counter's atomicAdd
//                      gives the pair's rank in the brick's list)
//     k_stats, k_offsets, k_fill_pairs   statistics, list offsets and work
//                      units (heavy bricks split), list fill
//     k_apply_brick    persistent: one workgroup owns one brick at a time in
//                      LDS, stamps the eq. 3 masks of every listed point with
//                      LDS atomicAnd (eq. 4) and counts shadow hits with LDS
//                      atomicAdd, then merges the brick into HBM once:
//                      mask &= stamp (write skipped when unchanged) and
//                      h = min(h + c, H_max) with the eq. 6 sign rule
//   k_download the statistics counters into the ring slot (per brick)
//
// Merging per brick is exact because the eq. 4 AND commutes and is
// idempotent, and c unit steps of eq. 5 saturate to min(h + c, H_max) while
// eq. 6 clears the sign iff h_old < T <= h_new; so the grid does not depend on
// the order of points or scans.
//
// Nothing here is a dense contraction, so MFMA is not used; the bound is HBM
// and L2/LDS atomic throughput.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>

#include "internal.h"

namespace dbtsdf {

// ============================================================== helpers ===
__device__ __forceinline__ uint32_t lane() { return __lane_id(); }

// Voxel planes are device memory. Reaching them through global-address-space
// pointers makes the compiler emit global_* rather than flat_* instructions;
// flat loads also count against the LDS wait counter, so every LDS read
// after them would wait for the outstanding voxel loads too.
// A grid descriptor held in scalar registers (its fields are the same for
// the whole wavefront).
// (readfirstlane returns int: each half is taken as uint32_t before widening,
// or a low half with bit 31 set would sign-extend over the high half)
__device__ __forceinline__ uint64_t sgpr64(uint64_t v) {
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
    return ((uint64_t)hi << 32) | (uint64_t)lo;
}
__device__ __forceinline__ DevGrid uniform_grid(const DevGrid &in) {
    DevGrid g = in;
    g.mask = reinterpret_cast<uint32_t *>(sgpr64(reinterpret_cast<uint64_t>(in.mask)));
    g.packed = reinterpret_cast<uint32_t *>(sgpr64(reinterpret_cast<uint64_t>(in.packed)));
    g.nx = __builtin_amdgcn_readfirstlane(in.nx);
    g.ny = __builtin_amdgcn_readfirstlane(in.ny);
    g.nz = __builtin_amdgcn_readfirstlane(in.nz);
    g.T = __builtin_amdgcn_readfirstlane(in.T);
    g.hmax = __builtin_amdgcn_readfirstlane(in.hmax);
    return g;
}

typedef __attribute__((address_space(1))) uint32_t gu32;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 gu32x4;
__device__ __forceinline__ gu32 *glob(uint32_t *p) { return (gu32 *)p; }
__device__ __forceinline__ uint4 gload4(const uint4 *p, size_t i) {
    const u32x4 v = ((gu32x4 *)p)[i];
    return make_uint4(v[0], v[1], v[2], v[3]);
}
// A 16-byte store to global memory. Pointers read from memory (the grid
// descriptors) are generic to the compiler; a generic (flat) access also
// counts against the LDS wait counter, so every later LDS wait would wait for
// it too.
__device__ __forceinline__ void gstore4(uint32_t *p, uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3) {
    typedef __attribute__((address_space(1))) u32x4 gu32x4w;
    u32x4 v;
    v[0] = a0;
    v[1] = a1;
    v[2] = a2;
    v[3] = a3;
    *reinterpret_cast<gu32x4w *>(glob(p)) = v;
}
__device__ __forceinline__ void g_and(gu32 *p, uint32_t v) {
    (void)__hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t g_add(gu32 *p, uint32_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t g_cas(gu32 *p, uint32_t expected, uint32_t desired) {
    (void)__hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
    return expected;   // the value found (equal to the one expected when the exchange took place)
}
typedef __attribute__((address_space(1))) const float gf32;
__device__ __forceinline__ gf32 *globf(const float *p) { return (gf32 *)p; }
__device__ __forceinline__ void g_sub(gu32 *p, uint32_t v) {
    (void)__hip_atomic_fetch_sub(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
    const uint32_t l = lane();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (l >= (uint32_t)o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t popc_below(unsigned long long m) {
    const uint32_t l = lane();
    unsigned long long below = l == 0 ? 0ull : (m & ((1ull << l) - 1ull));
    return (uint32_t)__popcll(below);
}

// Adds val into ctr[key * SC_N + field], one atomic per distinct key in the
// wave. Every lane of the wave must call it (uniform control flow).
__device__ __forceinline__ void wave_add(unsigned long long *ctr, uint32_t key, uint32_t field, uint32_t val) {
    unsigned long long pending = __ballot(val != 0u);
    while (pending) {
        const uint32_t leader = (uint32_t)__builtin_ctzll(pending);
        const uint32_t k0 = __shfl(key, leader, 64);
        const bool mine = val != 0u && key == k0;
        const uint32_t sum = wave_sum_u32(mine ? val : 0u);
        if (lane() == leader) atomicAdd(&ctr[(size_t)k0 * SC_N + field], (unsigned long long)sum);
        pending &= ~__ballot(mine);
    }
}

// Claims consecutive slots of *counter for the lanes with want = true (one
// atomic per wave); returns the lane's slot (undefined when !want).
__device__ __forceinline__ uint32_t wave_claim(uint32_t *counter, bool want) {
    const unsigned long long m = __ballot(want);
    uint32_t base = 0;
    if (m) {
        const uint32_t leader = (uint32_t)__builtin_ctzll(m);
        if (lane() == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
        base = __shfl(base, leader, 64);
    }
    return base + popc_below(m);
}

__device__ __forceinline__ uint32_t find_scan(const DevScan *scans, uint32_t n_scans, uint32_t i) {
    uint32_t lo = 0, hi = n_scans;  // largest s with scans[s].begin <= i
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (scans[mid].begin <= i) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t hash_of(unsigned long long k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return (uint32_t)k;
}

// ===================================================== front end (III-C) ===
// fp32, one IEEE operation per statement (the library is built with
// -ffp-contract=off and denormals kept).
__device__ __forceinline__ int bin_cube26(float dx, float dy, float dz) {
    const float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
    const float m = fmaxf(ax, fmaxf(ay, az));
    const float lim = 0.414213562373095f * m;
    const int sx = ax >= lim ? (dx > 0.0f ? 1 : -1) : 0;
    const int sy = ay >= lim ? (dy > 0.0f ? 1 : -1) : 0;
    const int sz = az >= lim ? (dz > 0.0f ? 1 : -1) : 0;
    const int code = (sx + 1) * 9 + (sy + 1) * 3 + (sz + 1);
    return code - (code > 13 ? 1 : 0);
}

__device__ __forceinline__ int bin_azel(const DevTables &t, float dx, float dy, float dz) {
    const int baz = (int)t.bins_az, bel = (int)t.bins_el;
    int b_az = 0;
    if (dx != 0.0f || dy != 0.0f) {
        const bool lower = dy < 0.0f || (dy == 0.0f && dx < 0.0f);
        const float ux = lower ? -dx : dx, uy = lower ? -dy : dy;
        int c = 0;
        for (int k = 1; k < baz / 2; ++k) {
            const float l = t.az_c[k] * uy;
            const float r = t.az_s[k] * ux;
            c += (l - r) >= 0.0f;
        }
        b_az = (lower ? baz / 2 : 0) + c;
    }
    const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
    const float q = (xx + yy) + zz;
    const bool up = dz >= 0.0f;
    int b_el = 0;
    for (int k = 1; k < bel; ++k) {
        const float rhs = t.el_s2[k] * q;
        b_el += t.el_neg[k] ? (up || zz <= rhs) : (up && zz >= rhs);
    }
    return b_el * baz + b_az;
}

// The pose of a return at time fraction tau of a motion-compensated sweep
// (Sec. III-C): the normalised linear interpolation between the identity and
// the sweep's rotation quaternion q, as the rotation matrix of a quaternion
// of any length (2 / |p|^2 in place of 2), applied after the start rotation;
// the translation moves linearly. fp32, one operation at a time.
__device__ __forceinline__ void sweep_pose(const DevScan &s, float tau, float rot[9], float tr[3]) {
    const float a = 1.0f - tau;
    const float qw = tau * s.dq[0];
    const float w = a + qw, x = tau * s.dq[1], y = tau * s.dq[2], z = tau * s.dq[3];
    const float ww = w * w, xx = x * x, yy = y * y, zz = z * z;
    const float wx = w * x, wy = w * y, wz = w * z, xy = x * y, xz = x * z, yz = y * z;
    const float n2 = ((ww + xx) + yy) + zz;
    const float s2 = 2.0f / n2;
    float m[9];
    m[0] = 1.0f - s2 * (yy + zz);
    m[1] = s2 * (xy - wz);
    m[2] = s2 * (xz + wy);
    m[3] = s2 * (xy + wz);
    m[4] = 1.0f - s2 * (xx + zz);
    m[5] = s2 * (yz - wx);
    m[6] = s2 * (xz - wy);
    m[7] = s2 * (yz + wx);
    m[8] = 1.0f - s2 * (xx + yy);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const float u = m[3 * i + 0] * s.rot[j];
            const float v = m[3 * i + 1] * s.rot[3 + j];
            const float e = m[3 * i + 2] * s.rot[6 + j];
            const float uv = u + v;
            rot[3 * i + j] = uv + e;
        }
        const float step = tau * s.dt[i];
        tr[i] = s.trans[i] + step;
    }
}

__device__ __forceinline__ uint32_t front_end(const DevScan &s, const DevGrid &g, const DevTables &t, float px,
                                              float py, float pz, bool deskew, float tau, int &vx, int &vy, int &vz,
                                              int &bin) {
    if (!__builtin_isfinite(px) || !__builtin_isfinite(py) || !__builtin_isfinite(pz)) return kStInvalid;
    float rot[9], tr[3];
    if (deskew) {
        if (!(tau >= 0.0f && tau <= 1.0f)) return kStInvalid;
        sweep_pose(s, tau, rot, tr);
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) rot[k] = s.rot[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) tr[k] = s.trans[k];
    }
    float d[3], w[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float a = rot[3 * k + 0] * px;
        const float b = rot[3 * k + 1] * py;
        const float c = rot[3 * k + 2] * pz;
        const float ab = a + b;
        d[k] = ab + c;
        w[k] = d[k] + tr[k];
    }
    if (d[0] == 0.0f && d[1] == 0.0f && d[2] == 0.0f) return kStInvalid;
    const uint32_t dims[3] = {g.nx, g.ny, g.nz};
    int v[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float rel = w[k] - s.origin[k];
        const float f = floorf(rel * s.inv_s);
        const float lo = (float)t.R;
        const float hi = (float)((int)dims[k] - 1 - t.R);
        if (!(f >= lo && f <= hi)) return kStOob;
        v[k] = (int)f;
    }
    vx = v[0];
    vy = v[1];
    vz = v[2];
    bin = t.binning == DBTSDF_BIN_CUBE26 ? bin_cube26(d[0], d[1], d[2]) : bin_azel(t, d[0], d[1], d[2]);
    return kStOk;
}

// ================================================================ passes ===
constexpr int kPtThreads = 256;
constexpr int kSelThreads = 256;    // one claim atomic per block of points

constexpr uint32_t kCtrlWords = sizeof(Ctrl) / 4;

// Clears the call's counters: threads [first, first + stride) of the launch.
// keep_active: leave Ctrl::n_active (word 0) alone.
__device__ __forceinline__ void reset_counters(const PipeArgs &a, uint32_t n_scans, uint32_t n_grids, uint32_t first,
                                               uint32_t stride, bool keep_active = false) {
    const uint32_t n_sc = n_scans * SC_N, n_tc = n_grids * TC_N;
    for (uint32_t i = first; i < n_sc + n_tc + kCtrlWords; i += stride) {
        if (i < n_sc) a.scan_ctr[i] = 0ull;
        else if (i < n_sc + n_tc) a.traffic_ctr[i - n_sc] = 0ull;
        else if (!keep_active || i != n_sc + n_tc) ((uint32_t *)a.ctrl)[i - n_sc - n_tc] = 0u;
    }
}

__global__ void k_reset(PipeArgs a, const CallInfo *info) {
    reset_counters(a, info->n_scans, info->n_grids, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

// First pass of a call: the descriptors, from the ring slot's pinned host
// buffer into device memory (ctrl + 1).
constexpr int kCopyBlocks = 16;
__global__ __launch_bounds__(256) void k_upload(PipeArgs a) {
    const uint32_t n_sc = reinterpret_cast<const CallInfo *>(a.host_desc)->n_scans;
    const uint32_t words = (a.desc_scans_off + n_sc * (uint32_t)sizeof(DevScan)) / 8u;
    uint2 *dst = reinterpret_cast<uint2 *>(a.ctrl + 1);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x)
        dst[i] = a.host_desc[i];
}

// Last pass of a call: the statistics counters into the ring slot's pinned
// host buffer.
__global__ __launch_bounds__(256) void k_download(PipeArgs a, const CallInfo *info) {
    const uint32_t n_s = info->n_scans * SC_N, n_t = info->n_grids * TC_N;
    // the tile strategy's one-scan front pass counts on a cleared work-item
    // counter (the brick passes that read it are done)
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctrl->n_active = 0u;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_s + n_t; i += gridDim.x * blockDim.x) {
        if (i < n_s) a.host_ctr[i] = a.scan_ctr[i];
        else a.host_ctr[(size_t)a.scans_cap * SC_N + (i - n_s)] = a.traffic_ctr[i - n_s];
    }
    __threadfence_system();
}

// A workgroup barrier that orders LDS only: it waits for this wave's LDS
// operations, not for its global loads (__syncthreads' fence waits for every
// outstanding vector memory operation, which would drain loads issued ahead
// to overlap later work).
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Exclusive prefix of v over the block; *total receives the block sum.
// LDS_ONLY: the barriers order LDS only (see lds_barrier).
template <int THREADS, bool LDS_ONLY = false>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_tmp, uint32_t &total) {
    const uint32_t w = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan_u32(v);
    if (lane() == 63u) s_tmp[w] = incl;
    if constexpr (LDS_ONLY) lds_barrier(); else __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < THREADS / 64; ++k) {
        const uint32_t x = s_tmp[k];
        before += (uint32_t)k < w ? x : 0u;
        tot += x;
    }
    if constexpr (LDS_ONLY) lds_barrier(); else __syncthreads();
    total = tot;
    return before + incl - v;
}

// atomics issued together per return (list ranks)
constexpr int kSelUnroll = 6;
constexpr int kFrontUnroll = 12;   // the tile strategy: every list of a K = 11 window at once

// Transform, voxelise, bin and dedup-insert every point of the call. In a
// one-scan call (ONE) the passes that copy the descriptors in and clear the
// counters are folded in: every workgroup reads what it needs of the call's
// descriptors (the sizes, the grid, the scan) straight from the ring slot's
// pinned host buffer into LDS, in 16-byte reads issued together, and
// workgroup 0 also writes the whole device copy that the later passes read
// and clears the counters (no pass before this one touches either).
// TILE (the tile strategy): every valid return is also listed, before the
// survivor test, in each grid tile (kTileX x kTileY x kTileZ) its eq. 4 window
// reaches, or, for a return whose voxel an earlier call integrated (its
// window is skipped), each tile its shadow ball reaches: the atomicAdd on the
// tile's counter gives the return's rank in that tile's list, and the return
// that opens a tile claims its work item (one global atomic per workgroup).
constexpr uint32_t kInfoWords = sizeof(CallInfo) / 8, kGridWords = sizeof(DevGrid) / 8,
                   kScanWords = sizeof(DevScan) / 8;
constexpr uint32_t kOneDescWords = kInfoWords + kGridWords + kScanWords;
static_assert(kOneDescWords <= 64 && kCtrlWords + SC_N + TC_N <= (uint32_t)kPtThreads - 128, "one pass of workgroup 0");
constexpr uint32_t kScanPieces = sizeof(DevScan) / 16;
constexpr uint32_t kGridPieces = (sizeof(DevGrid) + 15) / 16;
static_assert(sizeof(CallInfo) == 16 && sizeof(DevScan) % 16 == 0 && 1 + kGridPieces + kScanPieces <= 64,
              "the one-scan front pass reads the descriptors in these 16-byte pieces");

// Shadow ball radius in voxels (the largest r with r^2 <= r_s^2), clipped to
// the kernel radius; -1 without a shadow.
__device__ __forceinline__ int shadow_extent(const DevTables &t) {
    if (t.shadow_r2 < 0) return -1;
    int rs = 0;
    while (rs < t.R && (rs + 1) * (rs + 1) <= t.shadow_r2) ++rs;
    return rs;
}

// The tiles a return's list entries go to: those its window (extent R) or,
// for a revisit, its shadow ball reaches, as a box of tile coordinates.
struct TileSpan {
    uint32_t x0, y0, z0, nx, ny, nz;   // first tile and tiles per axis (nx = 0: none)
};
__device__ __forceinline__ TileSpan tile_span(uint32_t vx, uint32_t vy, uint32_t vz, int ext) {
    TileSpan sp{0u, 0u, 0u, 0u, 0u, 0u};
    if (ext < 0) return sp;
    const uint32_t e = (uint32_t)ext;   // vx, vy, vz >= R >= ext (the bounds rule)
    sp.x0 = (vx - e) / kTileX;
    sp.y0 = (vy - e) / kTileY;
    sp.z0 = (vz - e) / kTileZ;
    sp.nx = (vx + e) / kTileX - sp.x0 + 1u;
    sp.ny = (vy + e) / kTileY - sp.y0 + 1u;
    sp.nz = (vz + e) / kTileZ - sp.z0 + 1u;
    return sp;
}
// The tile strategy's counter of tile id: the per-grid counter arrays hold a
// power of two of entries, indexed by id times an odd constant modulo that
// size (a bijection), so that the counters of neighbouring tiles, which the
// returns of one neighbourhood update together, lie on different cache lines.
__device__ __forceinline__ uint32_t tile_ctr(const DevGrid &g, uint32_t id) {
    const unsigned long long n = (unsigned long long)g.nbx * g.nby * g.nbz;
    const unsigned long long cap = n <= 1ull ? 1ull : 1ull << (64 - __clzll(n - 1ull));
    return (uint32_t)((id * 0x9E3779B1u) & (uint32_t)(cap - 1ull));
}
__device__ __forceinline__ uint32_t span_tile(const TileSpan &sp, uint32_t j, const DevGrid &g) {
    const uint32_t jx = j % sp.nx, jy = (j / sp.nx) % sp.ny, jz = j / (sp.nx * sp.ny);
    return (sp.x0 + jx) + g.nbx * ((sp.y0 + jy) + g.nby * (sp.z0 + jz));
}

// The tile strategy's list counts, aggregated per workgroup: a table in LDS
// keyed by (grid, tile counter) counts the workgroup's lists of each tile
// (the add's old value is the list's rank within the workgroup), then one
// global atomic per distinct tile reserves the workgroup's run of ranks.
// Global atomics are the scarce resource (some 25 G/s over the whole device
// for scattered addresses); a list whose key does not find a slot within the
// probe limit, or whose grid index is 15 or more, takes its rank from the
// global counter directly (every rank is still a distinct reservation).
constexpr uint32_t kTileAggSlots = 2048;   // >= 2/3 of a workgroup's at most 256 x 12 lists
constexpr uint32_t kTileAggProbes = 16;
static_assert(kTileAggSlots == 1u << 11, "the slot hash takes the top 11 bits");

template <bool ONE, bool TILE>
__global__ __launch_bounds__(kPtThreads) void k_front(PipeArgs a, const CallInfo *info_dev) {
    __shared__ uint4 s_desc[ONE ? 1 + kGridPieces + kScanPieces : 1];
    __shared__ uint32_t s_tmp[kPtThreads / 64];
    __shared__ uint32_t s_base;
    __shared__ uint32_t s_akey[TILE ? kTileAggSlots : 1];   // (grid << 28 | counter) + 1; 0: empty
    __shared__ uint32_t s_acnt[TILE ? kTileAggSlots : 1];   // lists of the workgroup, then the reserved base
    const CallInfo *info = info_dev;
    const DevScan *scans = a.scans;
    const DevGrid *grids = a.grids;
    if constexpr (ONE) {
        const uint32_t t = threadIdx.x;
        // host layout: CallInfo, DevGrid[grids_cap] (16-byte pieces 1 on) and,
        // at desc_scans_off (a multiple of 16), DevScan[n_scans]
        const uint4 *h16 = reinterpret_cast<const uint4 *>(a.host_desc);
        if (t < 1u + kGridPieces + kScanPieces)
            s_desc[t] = h16[t <= kGridPieces ? t : a.desc_scans_off / 16u + (t - 1u - kGridPieces)];
        if (blockIdx.x == 0) {
            if (t >= 64u && t < 64u + kOneDescWords) {
                const uint32_t w = t - 64u;
                const uint32_t src = w < kInfoWords + kGridWords ? w : a.desc_scans_off / 8u + (w - kInfoWords - kGridWords);
                reinterpret_cast<uint2 *>(a.ctrl + 1)[src] = a.host_desc[src];
            } else if (t >= 128u) {
                // the tile strategy's work-item counter is in use by this pass:
                // the select pass of the previous call cleared it
                reset_counters(a, 1u, 1u, t - 128u, kPtThreads - 128u, TILE);
            }
        }
        __syncthreads();
        info = reinterpret_cast<const CallInfo *>(s_desc);
        grids = reinterpret_cast<const DevGrid *>(s_desc + 1);
        scans = reinterpret_cast<const DevScan *>(s_desc + 1 + kGridPieces);
    }
    const uint32_t n = info->n_points, n_scans = info->n_scans;
    const int R = a.tab.R;
    const int rs = TILE ? shadow_extent(a.tab) : 0;
    // block-uniform rounds (the tile claims synchronise the workgroup)
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        uint32_t n_open = 0, gi = 0, np = 0;
        unsigned long long opened = 0;   // list j of the return opened its tile
        TileSpan sp{0u, 0u, 0u, 0u, 0u, 0u};
        if constexpr (TILE) {
            for (uint32_t q = threadIdx.x; q < kTileAggSlots; q += kPtThreads) {
                s_akey[q] = 0u;
                s_acnt[q] = 0u;
            }
            __syncthreads();
        }
        if (i < n) {
            const uint32_t s = ONE ? 0u : find_scan(scans, n_scans, i);
            const DevScan &sc = scans[s];
            gi = ONE ? 0u : sc.grid;
            const DevGrid &g = grids[gi];
            const uint32_t j = i - sc.begin;
            const gf32 *pp = globf(sc.pts) + 3 * (size_t)j * sc.step;
            const float px = pp[0];
            const float py = pp[1];
            const float pz = pp[2];
            const bool deskew = sc.deskew != 0u;
            const float tau = deskew ? globf(sc.times)[(size_t)j * sc.step] : 0.0f;
            int vx = 0, vy = 0, vz = 0, bin = 0;
            const uint32_t st = front_end(sc, g, a.tab, px, py, pz, deskew, tau, vx, vy, vz, bin);
            uint32_t slot = kNoSlot;
            const unsigned long long lin = (unsigned long long)vx +
                (unsigned long long)g.nx * ((unsigned long long)vy + (unsigned long long)g.ny * (unsigned long long)vz);
            if (st == kStOk && sc.dedup) {
                const unsigned long long key = ((unsigned long long)s << kVoxelKeyBits) | lin;
                uint32_t h = hash_of(key) & a.hash_mask;
                for (;;) {  // the table holds >= 2x the call's points, so an empty slot exists
                    const unsigned long long prev = atomicCAS(&a.hkeys[h], kHashEmpty, key);
                    if (prev == kHashEmpty || prev == key) {
                        atomicMin(&a.hvals[h], i);
                        break;
                    }
                    h = (h + 1) & a.hash_mask;
                }
                slot = h;
            }
            uint32_t w = (st << 16) | (uint32_t)bin;
            if constexpr (TILE) {
                if (st == kStOk) {
                    // a return in a voxel an earlier call integrated (mask 0)
                    // skips its window: its lists are those of its shadow
                    const bool rv = a.revisit_ok && g.revisit_skip && glob(g.mask)[lin] == 0u;
                    if (rv) w |= kRecTileRevisit;
                    sp = tile_span((uint32_t)vx, (uint32_t)vy, (uint32_t)vz, rv ? rs : R);
                    np = sp.nx * sp.ny * sp.nz;   // at most 2 x 2 x 3 for K <= 11
                }
            }
            a.rec[i] = make_uint4((uint32_t)vx, (uint32_t)vy, (uint32_t)vz, w);
            a.pslot[i] = slot;
        }
        if constexpr (TILE) {
            // each list: its slot in the workgroup's table and its rank among
            // the workgroup's lists of the tile, or (no slot) its global rank
            const DevGrid &g = grids[gi];
            uint32_t ctr[kFrontUnroll], loc[kFrontUnroll];
#pragma unroll
            for (int u = 0; u < kFrontUnroll; ++u) {
                ctr[u] = 0u;
                loc[u] = 0u;
                if ((uint32_t)u >= np) continue;
                ctr[u] = tile_ctr(g, span_tile(sp, (uint32_t)u, g));
                bool placed = false;
                if (gi < 15u && ctr[u] < (1u << 28)) {
                    const uint32_t key = ((gi << 28) | ctr[u]) + 1u;
                    uint32_t h = (key * 0x9E3779B1u) >> (32 - 11);   // 11 bits: kTileAggSlots
                    for (uint32_t p = 0; p < kTileAggProbes; ++p, h = (h + 1u) & (kTileAggSlots - 1u)) {
                        const uint32_t prev = atomicCAS(&s_akey[h], 0u, key);
                        if (prev == 0u || prev == key) {
                            loc[u] = (h << 16) | atomicAdd(&s_acnt[h], 1u);   // at most 3072 lists: 12 bits
                            placed = true;
                            break;
                        }
                    }
                }
                if (!placed) loc[u] = 0x80000000u | g_add(glob(g.brick_cnt) + ctr[u], 1u);
            }
            __syncthreads();
            // one global atomic per distinct tile of the workgroup
            for (uint32_t q = threadIdx.x; q < kTileAggSlots; q += kPtThreads) {
                const uint32_t key = s_akey[q];
                if (key) {
                    const uint32_t kk = key - 1u, kg = kk >> 28;
                    s_acnt[q] = g_add(glob(grids[kg].brick_cnt) + (kk & 0x0FFFFFFFu), s_acnt[q]);
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kFrontUnroll; ++u) {
                if ((uint32_t)u >= np) continue;
                const uint32_t rk = (loc[u] & 0x80000000u) ? (loc[u] & 0x7FFFFFFFu)
                                                           : s_acnt[loc[u] >> 16] + (loc[u] & 0xFFFFu);
                // list j's rank at j n + i (a wavefront's stores contiguous)
                a.rank[(size_t)u * n + i] = rk;
                if (rk == 0u) {
                    ++n_open;
                    opened |= 1ull << u;
                }
            }
        }
        if constexpr (TILE) {
            uint32_t total;
            const uint32_t pos = block_excl_scan<kPtThreads>(n_open, s_tmp, total);
            if (total) {
                if (threadIdx.x == 0) s_base = atomicAdd(&a.ctrl->n_active, total);
                __syncthreads();
                if (n_open) {
                    const DevGrid &g = grids[gi];
                    uint32_t k = 0;
                    for (uint32_t j = 0; j < 64u && opened; ++j) {
                        if (!((opened >> j) & 1ull)) continue;
                        opened &= ~(1ull << j);
                        const uint32_t id = span_tile(sp, j, g);
                        const uint32_t slot = s_base + pos + k++;
                        a.items[slot] = ((unsigned long long)gi << 32) | id;
                    }
                }
                __syncthreads();  // s_base is reused by the next round
            }
        }
    }
}

struct SelectOut {
    bool surv;
    bool dup;
    uint32_t s;
    uint32_t shadow_n;
    uint4 r;
};

__device__ __forceinline__ SelectOut select_point(const PipeArgs &a, const CallInfo *info, uint32_t i, bool live) {
    SelectOut o{false, false, 0u, 0u, make_uint4(0, 0, 0, 0)};
    if (!live) return o;
    o.r = a.rec[i];
    if (((o.r.w >> 16) & 3u) != kStOk) return o;  // bits 16-17 only: bit 30 may already be set
    o.s = find_scan(a.scans, info->n_scans, i);
    const DevScan &sc = a.scans[o.s];
    o.surv = !sc.dedup || a.hvals[a.pslot[i]] == i;
    o.dup = !o.surv;
    if (o.surv) {
        const uint32_t bin = o.r.w & 0xFFFFu;
        o.shadow_n = a.tab.sh_start[bin + 1] - a.tab.sh_start[bin];
    }
    return o;
}

// brick j of the (at most span[0] x span[1] x span[2]) bricks a K^3 cube touches
__device__ __forceinline__ bool pair_brick(const PipeArgs &a, const uint4 &r, uint32_t j, const DevGrid &g,
                                           uint32_t &id) {
    const int R = a.tab.R;
    const uint32_t mx = a.span[0], my = a.span[1];
    const uint32_t jx = j % mx, jy = (j / mx) % my, jz = j / (mx * my);
    const uint32_t bx = (r.x - (uint32_t)R) / a.brick[0] + jx;
    const uint32_t by = (r.y - (uint32_t)R) / a.brick[1] + jy;
    const uint32_t bz = (r.z - (uint32_t)R) / a.brick[2] + jz;
    if (bx > (r.x + (uint32_t)R) / a.brick[0] || by > (r.y + (uint32_t)R) / a.brick[1] ||
        bz > (r.z + (uint32_t)R) / a.brick[2])
        return false;
    id = bx + g.nbx * (by + g.nby * bz);
    return true;
}

// One thread per point: the survivor test, then one atomicAdd per brick its
// K^3 cube touches on that brick's counter (issued kSelUnroll at a time so
// that they are in flight together); the returned old count is the pair's
// rank in the brick's list. Pairs that open a brick take work-item slots,
// one global atomic per block.

__global__ __launch_bounds__(kSelThreads) void k_select_pairs(PipeArgs a, const CallInfo *info) {
    __shared__ uint32_t s_tmp[kSelThreads / 64];
    __shared__ uint32_t s_base;
    const uint32_t n = info->n_points;
    const uint32_t F = a.span[0] * a.span[1] * a.span[2];
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        const SelectOut o = select_point(a, info, i, i < n);
        unsigned long long opened_bits = 0;   // pair j opened its brick (j < 64)
        uint32_t n_open = 0, gi = 0;
        DevGrid g{};
        if (o.surv) {
            a.rec[i].w = o.r.w | kRecSurvivor;
            gi = a.scans[o.s].grid;
            g = a.grids[gi];
            for (uint32_t j0 = 0; j0 < F; j0 += kSelUnroll) {
                uint32_t rk[kSelUnroll];
                bool v[kSelUnroll];
#pragma unroll
                for (int u = 0; u < kSelUnroll; ++u) {
                    uint32_t id = 0;
                    v[u] = j0 + u < F && pair_brick(a, o.r, j0 + u, g, id);
                    rk[u] = v[u] ? g_add(glob(g.brick_cnt) + id, 1u) : 1u;
                }
#pragma unroll
                for (int u = 0; u < kSelUnroll; ++u) {
                    if (!v[u]) continue;
                    a.rank[(size_t)i * F + j0 + u] = rk[u];
                    if (rk[u] == 0u) {
                        ++n_open;
                        if (j0 + u < 64) opened_bits |= 1ull << (j0 + u);
                    }
                }
            }
        }
        uint32_t total;
        const uint32_t pos = block_excl_scan<kSelThreads>(n_open, s_tmp, total);
        if (total) {
            if (threadIdx.x == 0) s_base = atomicAdd(&a.ctrl->n_active, total);
            __syncthreads();
            uint32_t k = 0;
            for (uint32_t j = 0; j < F && k < n_open; ++j) {
                const bool op = j < 64 ? ((opened_bits >> j) & 1ull) != 0ull : a.rank[(size_t)i * F + j] == 0u;
                uint32_t id = 0;
                if (!op || !pair_brick(a, o.r, j, g, id)) continue;
                const uint32_t slot = s_base + pos + k++;
                a.items[slot] = ((unsigned long long)gi << 32) | id;
                glob(g.brick_slot)[id] = slot;
            }
            __syncthreads();
        }
    }
}

// Per-scan statistics from the point records (after the select pass): each
// block reduces a contiguous run of points; a run inside one scan costs one
// atomic per counter.
__global__ __launch_bounds__(kPtThreads) void k_stats(PipeArgs a, const CallInfo *info, uint32_t chunk) {
    __shared__ uint32_t s_red[SC_N][kPtThreads / 64];
    const uint32_t n = info->n_points;
    for (uint32_t lo = blockIdx.x * chunk; lo < n; lo += gridDim.x * chunk) {
        const uint32_t hi = min(n, lo + chunk);
        const uint32_t s0 = find_scan(a.scans, info->n_scans, lo);
        const uint32_t s1 = find_scan(a.scans, info->n_scans, hi - 1);
        if (s0 == s1) {
            uint32_t c[SC_N] = {};
            for (uint32_t i = lo + threadIdx.x; i < hi; i += kPtThreads) {
                const uint32_t w = a.rec[i].w;
                const uint32_t st = (w >> 16) & 3u;
                c[SC_INVALID] += st == kStInvalid;
                c[SC_OOB] += st == kStOob;
                const bool surv = st == kStOk && (w & kRecSurvivor);
                c[SC_DUP] += st == kStOk && !surv;
                c[SC_INT] += surv;
                if (surv) c[SC_SHADOW] += a.tab.sh_start[(w & 0xFFFFu) + 1] - a.tab.sh_start[w & 0xFFFFu];
            }
#pragma unroll
            for (int f = 0; f < SC_N; ++f) {
                const uint32_t v = wave_sum_u32(c[f]);
                if (lane() == 0) s_red[f][threadIdx.x >> 6] = v;
            }
            __syncthreads();
            if (threadIdx.x < SC_N) {
                unsigned long long tot = 0;
                for (int k = 0; k < kPtThreads / 64; ++k) tot += s_red[threadIdx.x][k];
                if (tot) atomicAdd(&a.scan_ctr[(size_t)s0 * SC_N + threadIdx.x], tot);
            }
            __syncthreads();
        } else {
            for (uint32_t b0 = lo; b0 < hi; b0 += kPtThreads) {
                const uint32_t i = b0 + threadIdx.x;
                uint32_t w = 0, s = 0;
                if (i < hi) {
                    w = a.rec[i].w;
                    s = find_scan(a.scans, info->n_scans, i);
                }
                const uint32_t st = i < hi ? (w >> 16) & 3u : 3u;
                const bool surv = st == kStOk && (w & kRecSurvivor);
                wave_add(a.scan_ctr, s, SC_INVALID, st == kStInvalid);
                wave_add(a.scan_ctr, s, SC_OOB, st == kStOob);
                wave_add(a.scan_ctr, s, SC_DUP, st == kStOk && !surv);
                wave_add(a.scan_ctr, s, SC_INT, surv);
                wave_add(a.scan_ctr, s, SC_SHADOW,
                         surv ? a.tab.sh_start[(w & 0xFFFFu) + 1] - a.tab.sh_start[w & 0xFFFFu] : 0u);
            }
        }
    }
}

// Per touched brick: list offset (exclusive scan of the counts), count, and
// its apply work units (bricks with more than `chunk` listed points are split).
// Resets the brick counters for the next call.
__global__ __launch_bounds__(kPtThreads) void k_offsets(PipeArgs a) {
    __shared__ uint32_t s_tmp[kPtThreads / 64];
    __shared__ uint32_t s_bases[2];
    const uint32_t n = a.ctrl->n_active;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t t = base + threadIdx.x;
        uint32_t cnt = 0;
        if (t < n) {
            const unsigned long long it = a.items[t];
            const DevGrid &g = a.grids[it >> 32];
            gu32 *bc = glob(g.brick_cnt) + (a.tile_mode ? tile_ctr(g, (uint32_t)it) : (uint32_t)it);
            cnt = *bc;
            *bc = 0u;
        }
        // entry and work-unit offsets: one scan and one atomic per counter
        // per workgroup (same-address atomics queue at the coherence point)
        const uint32_t nsub = t < n ? (a.chunk ? (cnt + a.chunk - 1u) / a.chunk : 1u) : 0u;
        uint32_t tot_e, tot_s;
        const uint32_t ex = block_excl_scan<kPtThreads>(cnt, s_tmp, tot_e);
        const uint32_t sex = block_excl_scan<kPtThreads>(nsub, s_tmp, tot_s);
        if (threadIdx.x == 0) {
            s_bases[0] = tot_e ? atomicAdd(&a.ctrl->total_entries, tot_e) : 0u;
            s_bases[1] = tot_s ? atomicAdd(&a.ctrl->n_work, tot_s) : 0u;
        }
        __syncthreads();
        const uint32_t wbase = s_bases[0], sbase = s_bases[1];
        __syncthreads();   // s_bases is reused by the next round
        if (t < n) {
            const unsigned long long it = a.items[t];
            const uint32_t first = wbase + ex;
            const uint32_t sincl = sex + nsub;
            a.item_off[t] = first;
            a.item_cnt[t] = cnt;
            // the tile strategy's fill finds the list's first entry beside the counter
            if (a.tile_mode) {
                const DevGrid &g = a.grids[it >> 32];
                glob(g.brick_slot)[tile_ctr(g, (uint32_t)it)] = first;
            }
            const uint32_t split = nsub > 1u ? 0x80000000u : 0u;
            for (uint32_t k = 0; k < nsub; ++k) {
                const uint32_t s0 = a.chunk ? k * a.chunk : 0u;
                const uint32_t c0 = a.chunk ? min(a.chunk, cnt - s0) : cnt;
                a.work[sbase + sincl - nsub + k] = make_uint4((uint32_t)it, (uint32_t)(it >> 32), first + s0, c0 | split);
            }
        }
    }
}

// Writes every (point, brick) pair at its rank in the brick's list, and
// releases the dedup hash slots (every reader is done).
__global__ __launch_bounds__(kPtThreads) void k_fill_pairs(PipeArgs a, const CallInfo *info) {
    const uint32_t n = info->n_points;
    const uint32_t F = a.span[0] * a.span[1] * a.span[2];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint4 r = a.rec[i];
        const uint32_t slot = a.pslot[i];
        if (slot != kNoSlot) {
            a.hkeys[slot] = kHashEmpty;
            a.hvals[slot] = 0xFFFFFFFFu;
        }
        if (!(r.w & kRecSurvivor)) continue;
        const DevGrid &g = a.grids[a.scans[find_scan(a.scans, info->n_scans, i)].grid];
        for (uint32_t j0 = 0; j0 < F; j0 += kSelUnroll) {
            uint32_t item[kSelUnroll], rk[kSelUnroll];
            bool v[kSelUnroll];
#pragma unroll
            for (int u = 0; u < kSelUnroll; ++u) {  // independent loads, all in flight
                uint32_t id = 0;
                v[u] = j0 + u < F && pair_brick(a, r, j0 + u, g, id);
                item[u] = v[u] ? glob(g.brick_slot)[id] : 0u;
                rk[u] = v[u] ? a.rank[(size_t)i * F + j0 + u] : 0u;
            }
#pragma unroll
            for (int u = 0; u < kSelUnroll; ++u)
                if (v[u]) a.entries[a.item_off[item[u]] + rk[u]] = make_uint4(r.x, r.y, r.z, r.w & 0xFFFFu);
        }
    }
}

// --------------------------------------------------------------- apply ---
// One workgroup owns one brick (BX, BY, BZ) of one grid per work unit. LDS
// holds the brick widened by twice the kernel radius on both x sides (a listed
// point lies at most R outside the brick and its cube reaches R further, so a
// row of K cells is never cut), as two tiles: the AND-accumulated eq. 3 stamp and the
// shadow hit counts. The row pitch is odd so that 64 lanes on 64 different
// rows hit 64 different banks.
//   1. the work unit's listed points are staged in LDS with everything a row
//      needs precomputed (one cooperative load of the list and the records);
//   2. each lane of a wavefront takes one (y, z) row of one point's cube that
//      lies in the brick and ANDs its K masks into the tile (the masks of a
//      row depend on |dx| only, so R + 1 table reads serve K cells), then adds
//      the shadow cells of the row;
//   3. the brick interior is merged into HBM 16 bytes at a time, every load
//      issued before the stores: mask &= stamp (store skipped when unchanged),
//      h = min(h + count, H_max), sign cleared on the crossing (eq. 6). A brick
//      split over several work units merges with atomics instead.
constexpr int kStage = 512;
constexpr int kLutMax = 3 * (kMaxK / 2) * (kMaxK / 2) + 1;

// x extent of the tile: BX + 4R, made odd
constexpr int row_pitch(int bx, int r) { return (bx + 4 * r) | 1; }

// largest kernel radius whose two tiles fit in LDS next to the staging area
constexpr int kLdsForTiles = 160 * 1024 - kStage * 16 - kLutMax * 4 - 1024;
constexpr int max_radius(int bx, int by, int bz) {
    int r = kMaxK / 2;
    while (r > 0 && 2 * row_pitch(bx, r) * by * bz * 4 > kLdsForTiles) --r;
    return r;
}

template <int BX, int BY, int BZ, int THREADS, int RR>
__global__ __launch_bounds__(THREADS) void k_apply_brick(PipeArgs a) {
    // RR > 0: rows unrolled for that radius; RR = 0: any radius up to the
    // largest whose tiles fit (the tile is sized for that)
    constexpr int RM = RR > 0 ? RR : max_radius(BX, BY, BZ);
    if constexpr (RM <= max_radius(BX, BY, BZ)) {
    constexpr int PX = row_pitch(BX, RM);
    constexpr int HX = 2 * RM;                          // tile column of brick-local x = 0
    constexpr int TILE = PX * BY * BZ;
    constexpr int WAVES = THREADS / 64;
    constexpr int V = BX * BY * BZ;
    constexpr int NQ = V / (4 * THREADS);
    constexpr int NB = NQ < 4 ? NQ : 4;
    static_assert(V % (4 * THREADS) == 0, "brick volume must be a multiple of 4 x threads");
    static_assert(NQ % NB == 0, "quads per thread must split evenly");
    static_assert(TILE % 4 == 0, "tile must hold whole 16-byte quads");
    __shared__ __align__(16) uint32_t tmask[TILE];
    __shared__ __align__(16) uint32_t tcnt[TILE];
    __shared__ uint32_t lut[kLutMax];
    __shared__ uint4 ent[kStage];
    __shared__ uint32_t red[3 * WAVES];

    const DevTables &t = a.tab;
    for (uint32_t q = threadIdx.x; q < t.n_q; q += THREADS) lut[q] = t.mask_by_q[q];
    const int R = RR > 0 ? RR : t.R;
    const bool l1 = t.metric == DBTSDF_DIST_L1;
    // cube bins with the hemispherical shadow take it row by row from the
    // integer test; every other shadow (AZEL bins, cones) from the bin's list
    const bool cube = t.binning == DBTSDF_BIN_CUBE26 && t.shadow_model == DBTSDF_SHADOW_HEMISPHERE;
    const int r2 = t.shadow_r2;
    const uint32_t n_work = a.ctrl->n_work;
    const uint32_t w = threadIdx.x >> 6, l = lane();

    // shadow ball radius, clipped to the kernel window: rows with |dy|, |dz| <= rs
    // can hold shadow cells
    int rs = 0;
    while (r2 >= 0 && rs < R && (rs + 1) * (rs + 1) <= r2) ++rs;

    for (uint32_t wi = blockIdx.x; wi < n_work; wi += gridDim.x) {
        const uint4 wk = a.work[wi];
        const uint32_t brick = wk.x;
        const bool split = (wk.w >> 31) != 0u;
        const DevGrid g = a.grids[wk.y];
        const uint32_t bxi = brick % g.nbx, byi = (brick / g.nbx) % g.nby, bzi = brick / (g.nbx * g.nby);
        const int x0 = (int)bxi * BX, y0 = (int)byi * BY, z0 = (int)bzi * BZ;
        const uint32_t start = wk.z;
        const uint32_t cnt = wk.w & 0x7FFFFFFFu;

        // the merge's mask loads are issued now, so that staging and stamping
        // hide their latency
        const bool vec_x = (g.nx & 3u) == 0;
        uint4 pm[NQ];
        bool fastq[NQ];
        size_t linq[NQ];
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const int v = 4 * ((int)threadIdx.x + k * THREADS);
            const uint32_t gx = (uint32_t)(x0 + v % BX), gy = (uint32_t)(y0 + (v / BX) % BY),
                           gz = (uint32_t)(z0 + v / (BX * BY));
            linq[k] = (size_t)gx + (size_t)g.nx * ((size_t)gy + (size_t)g.ny * gz);
            fastq[k] = !split && vec_x && gx + 3u < g.nx && gy < g.ny && gz < g.nz;
            if (fastq[k]) pm[k] = gload4(reinterpret_cast<const uint4 *>(g.mask + linq[k]), 0);
        }

        for (int q = threadIdx.x; q < TILE / 4; q += THREADS) {
            reinterpret_cast<uint4 *>(tmask)[q] = make_uint4(~0u, ~0u, ~0u, ~0u);
            reinterpret_cast<uint4 *>(tcnt)[q] = make_uint4(0u, 0u, 0u, 0u);
        }
        for (uint32_t base = 0; base < cnt; base += kStage) {
            const uint32_t nb = min(cnt - base, (uint32_t)kStage);
            __syncthreads();  // tile init done / previous round's readers done
            for (uint32_t e = threadIdx.x; e < nb; e += THREADS) {
                const uint4 r = a.entries[start + base + e];
                const int lx = (int)r.x - x0, ly = (int)r.y - y0, lz = (int)r.z - z0;
                const int ya = max(ly - R, 0), yb = min(ly + R, BY - 1);
                const int za = max(lz - R, 0), zb = min(lz + R, BZ - 1);
                const uint32_t wy = (uint32_t)(yb - ya + 1), rows = wy * (uint32_t)(zb - za + 1);
                // x: tile column of the cube's first cell; y, z: first row and the point
                ent[e] = make_uint4((uint32_t)(lx - R + HX) | ((uint32_t)ya << 12) | ((uint32_t)za << 22),
                                    (uint32_t)(ly + 64) | ((uint32_t)(lz + 64) << 8) | (wy << 16) | (rows << 22),
                                    r.w, __float_as_uint(1.0f / (float)wy));
            }
            __syncthreads();
            for (uint32_t e = w; e < nb; e += WAVES) {
                // the entry is the same for the whole wavefront: decode it in scalars
                const uint4 env = ent[e];
                const uint32_t ex = __builtin_amdgcn_readfirstlane(env.x);
                const uint32_t ey = __builtin_amdgcn_readfirstlane(env.y);
                const uint32_t bin = __builtin_amdgcn_readfirstlane(env.z);
                const float rwy = __uint_as_float(__builtin_amdgcn_readfirstlane(env.w));
                const int cx = (int)(ex & 4095u), ya = (int)((ex >> 12) & 1023u), za = (int)(ex >> 22);
                const int ly = (int)(ey & 255u) - 64, lz = (int)((ey >> 8) & 255u) - 64;
                const uint32_t wy = (ey >> 16) & 63u, rows = ey >> 22;
                const int code = (int)bin + (bin >= 13u ? 1 : 0);
                const int sxv = code / 9 - 1, syv = (code / 3) % 3 - 1, szv = code % 3 - 1;
                for (uint32_t rr = l; rr < rows; rr += 64u) {
                    const uint32_t rz = (uint32_t)(((float)rr + 0.5f) * rwy);
                    const uint32_t ry = rr - rz * wy;
                    const int yy = ya + (int)ry, zz = za + (int)rz;
                    const int oy = yy - ly, oz = zz - lz;
                    const int c2 = oy * oy + oz * oz;
                    const int row = cx + PX * (yy + BY * zz);
                    if (!l1) {
                        if constexpr (RR > 0) {
                            uint32_t m[RR + 1];
#pragma unroll
                            for (int k = 0; k <= RR; ++k) m[k] = lut[c2 + k * k];
#pragma unroll
                            for (int k = 0; k < 2 * RR + 1; ++k) atomicAnd(&tmask[row + k], m[k < RR ? RR - k : k - RR]);
                        } else {
                            for (int k = 0; k < 2 * R + 1; ++k) {
                                const int ox = k - R;
                                atomicAnd(&tmask[row + k], lut[c2 + ox * ox]);
                            }
                        }
                    } else {
                        const int c1 = abs(oy) + abs(oz);
                        for (int k = 0; k < 2 * R + 1; ++k) atomicAnd(&tmask[row + k], lut[c1 + abs(k - R)]);
                    }
                }
                if (cube && r2 >= 0) {
                    // shadow: only the rows of the r_s ball, and only when the ball
                    // reaches into the brick
                    const int lxb = cx + R - HX;  // brick-local x of the point
                    const int sya = max(ly - rs, 0), syb = min(ly + rs, BY - 1);
                    const int sza = max(lz - rs, 0), szb = min(lz + rs, BZ - 1);
                    if (sya <= syb && sza <= szb && lxb - rs <= BX - 1 && lxb + rs >= 0) {
                        const int swy = syb - sya + 1;
                        const int srows = swy * (szb - sza + 1);
                        const float rsw = 1.0f / (float)swy;
                        for (int sr = (int)l; sr < srows; sr += 64) {
                            const int srz = (int)(((float)sr + 0.5f) * rsw);
                            const int yy = sya + (sr - srz * swy), zz = sza + srz;
                            const int oy = yy - ly, oz = zz - lz;
                            const int c2 = oy * oy + oz * oz;
                            if (c2 > r2) continue;
                            int m = 0;
                            while (m < R && (m + 1) * (m + 1) <= r2 - c2) ++m;
                            const int dyz = oy * syv + oz * szv;
                            int lo = -m, hi = m;
                            if (sxv > 0) lo = max(lo, -dyz);
                            else if (sxv < 0) hi = min(hi, dyz);
                            else if (dyz < 0) hi = lo - 1;
                            lo = max(lo, -lxb);
                            hi = min(hi, BX - 1 - lxb);
                            const int rowp = cx + R + PX * (yy + BY * zz);  // tile index of the point's column
                            for (int ox = lo; ox <= hi; ++ox) atomicAdd(&tcnt[rowp + ox], 1u);
                        }
                    }
                }
                if (!cube) {
                    // AZEL: the bin's shadow list, clipped to the brick in y and z
                    const int lxt = cx + R;  // tile column of the point
                    const uint32_t s0 = t.sh_start[bin], s1 = t.sh_start[bin + 1];
                    for (uint32_t j = s0 + l; j < s1; j += 64u) {
                        const uint32_t off = t.sh_off[j];
                        const int sx = lxt + (int)(off & 255u) - R;
                        const int sy = ly + (int)((off >> 8) & 255u) - R;
                        const int sz = lz + (int)((off >> 16) & 255u) - R;
                        if (sy >= 0 && sy < BY && sz >= 0 && sz < BZ) atomicAdd(&tcnt[sx + PX * (sy + BY * sz)], 1u);
                    }
                }
            }
        }
        __syncthreads();

        // merge the brick interior into HBM, NB quads in flight per thread
        uint32_t um = 0, cm = 0, us = 0;
#pragma unroll
        for (int k0 = 0; k0 < NQ; k0 += NB) {
            uint32_t sm[NB][4], sc[NB][4];
            uint4 om[NB], op[NB];
            size_t lin[NB];
            bool fast[NB], need_m[NB], need_c[NB];
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const int q = (int)threadIdx.x + (k0 + k) * THREADS;
                const int v = 4 * q;
                const int xl = v % BX, yl = (v / BX) % BY, zl = v / (BX * BY);
                const int tb = HX + xl + PX * (yl + BY * zl);
                bool any_m = false, any_c = false;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    sm[k][j] = tmask[tb + j];
                    sc[k][j] = tcnt[tb + j];
                    any_m |= sm[k][j] != 0xFFFFFFFFu;
                    any_c |= sc[k][j] != 0u;
                }
                need_m[k] = any_m;
                need_c[k] = any_c;
                lin[k] = linq[k0 + k];
                fast[k] = fastq[k0 + k];
                om[k] = pm[k0 + k];
                if (fast[k] && any_c) op[k] = gload4(reinterpret_cast<const uint4 *>(g.packed + lin[k]), 0);
            }
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                if (!need_m[k] && !need_c[k]) continue;
                if (fast[k]) {
                    if (need_m[k]) {
                        const uint32_t o[4] = {om[k].x, om[k].y, om[k].z, om[k].w};
                        uint32_t nw[4];
                        bool ch = false;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            nw[j] = o[j] & sm[k][j];
                            um += sm[k][j] != 0xFFFFFFFFu;
                            cm += nw[j] != o[j];
                            ch |= nw[j] != o[j];
                        }
                        if (ch) gstore4(g.mask + lin[k], nw[0], nw[1], nw[2], nw[3]);
                    }
                    if (need_c[k]) {
                        const uint32_t o[4] = {op[k].x, op[k].y, op[k].z, op[k].w};
                        uint32_t nw[4];
                        bool ch = false;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const uint32_t h0 = o[j] & 0xFFFFu;
                            const uint32_t h1 = min(h0 + sc[k][j], g.hmax);
                            const uint32_t sign = (h0 < g.T && h1 >= g.T) ? 0u : (o[j] & 0x80000000u);
                            nw[j] = sc[k][j] ? (sign | h1) : o[j];
                            us += sc[k][j] != 0u;
                            ch |= nw[j] != o[j];
                        }
                        if (ch) gstore4(g.packed + lin[k], nw[0], nw[1], nw[2], nw[3]);
                    }
                    continue;
                }
                const int v = 4 * ((int)threadIdx.x + (k0 + k) * THREADS);
                const uint32_t gx = (uint32_t)(x0 + v % BX), gy = (uint32_t)(y0 + (v / BX) % BY),
                               gz = (uint32_t)(z0 + v / (BX * BY));
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (gx + j >= g.nx || gy >= g.ny || gz >= g.nz) continue;
                    const size_t li = lin[k] + j;
                    if (!split) {
                        // grid edge or Nx not a multiple of 4: element by element
                        if (sm[k][j] != 0xFFFFFFFFu) {
                            const uint32_t old = glob(g.mask)[li];
                            const uint32_t nw = old & sm[k][j];
                            if (nw != old) {
                                glob(g.mask)[li] = nw;
                                ++cm;
                            }
                            ++um;
                        }
                        if (sc[k][j]) {
                            const uint32_t old = glob(g.packed)[li];
                            const uint32_t h0 = old & 0xFFFFu;
                            const uint32_t h1 = min(h0 + sc[k][j], g.hmax);
                            const uint32_t sign = (h0 < g.T && h1 >= g.T) ? 0u : (old & 0x80000000u);
                            const uint32_t nw = sign | h1;
                            if (nw != old) glob(g.packed)[li] = nw;
                            ++us;
                        }
                    } else {
                        // a split brick: other work units merge into the same words, so
                        // the mask uses atomicAnd and the counter a compare-and-swap loop
                        // (c steps of eq. 5 then d steps equal c + d steps, and eq. 6
                        // fires once on the crossing, so the merge order does not matter)
                        if (sm[k][j] != 0xFFFFFFFFu) {
                            const uint32_t old = glob(g.mask)[li];
                            if ((old & sm[k][j]) != old) g_and(glob(g.mask) + li, sm[k][j]);
                        }
                        if (sc[k][j]) {
                            uint32_t old = glob(g.packed)[li];
                            for (;;) {
                                const uint32_t h0 = old & 0xFFFFu;
                                const uint32_t h1 = min(h0 + sc[k][j], g.hmax);
                                const uint32_t sign = (h0 < g.T && h1 >= g.T) ? 0u : (old & 0x80000000u);
                                const uint32_t nw = sign | h1;
                                if (nw == old) break;
                                const uint32_t prev = g_cas(glob(g.packed) + li, old, nw);
                                if (prev == old) break;
                                old = prev;
                            }
                        }
                    }
                }
            }
        }
        if (a.count_traffic) {
            const uint32_t su = wave_sum_u32(um), sc2 = wave_sum_u32(cm), ss = wave_sum_u32(us);
            if (l == 0) {
                red[3 * w + 0] = su;
                red[3 * w + 1] = sc2;
                red[3 * w + 2] = ss;
            }
            __syncthreads();
            if (threadIdx.x < 3) {
                unsigned long long tot = 0;
                for (int k = 0; k < WAVES; ++k) tot += red[3 * k + threadIdx.x];
                if (tot) atomicAdd(&a.traffic_ctr[(size_t)g.traffic_slot * TC_N + threadIdx.x], tot);
            }
        }
        __syncthreads();
    }
    }
}

// The call's statistics into the ring slot's pinned host buffer, by
// workgroup 0 of the apply pass: the counting passes have finished (stream
// order), and their counters are touched only by device-scope atomics. (A
// last-workgroup count in the counting pass instead would put one returning
// atomic per workgroup on one address, and those queue behind each other at
// the coherence point: 50-60 us for 1024 workgroups.)
__device__ void stats_out(const PipeArgs &a, const CallInfo *info) {
    const uint32_t n_s = info->n_scans * SC_N, n_t = info->n_grids * TC_N;
    for (uint32_t i = threadIdx.x; i < n_s + n_t; i += blockDim.x) {
        unsigned long long *src = i < n_s ? &a.scan_ctr[i] : &a.traffic_ctr[i - n_s];
        a.host_ctr[i < n_s ? (size_t)i : (size_t)a.scans_cap * SC_N + (i - n_s)] =
            __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");  // system scope: the host reads them
}

// ------------------------------------------------------ atomic strategy ---
// Per-point strategy, one pass per point before the apply: survivor test,
// compaction of the survivors into a list, the per-scan statistics, and the
// release of the point's dedup hash slot. Only the slot's winner (the point
// whose index the slot holds) releases it; a loser that reads the slot after
// the release sees the empty value, which is not its index either, so its
// answer is the same.
__global__ __launch_bounds__(kSelThreads) void k_select_atomic(PipeArgs a, const CallInfo *info) {
    __shared__ uint32_t s_tmp[kSelThreads / 64];
    __shared__ uint32_t s_base;
    __shared__ uint32_t s_red[SC_N][kSelThreads / 64];
    const uint32_t n = info->n_points;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        const bool live = i < n;
        uint4 r = make_uint4(0u, 0u, 0u, 0u);
        uint32_t s = 0, st = 3u;
        bool surv = false;
        if (live) {
            r = a.rec[i];
            st = (r.w >> 16) & 3u;
            s = find_scan(a.scans, info->n_scans, i);
            if (st == kStOk) {
                if (a.scans[s].dedup) {
                    const uint32_t slot = a.pslot[i];
                    surv = a.hvals[slot] == i;
                    if (surv) {
                        a.hkeys[slot] = kHashEmpty;
                        a.hvals[slot] = 0xFFFFFFFFu;
                    }
                } else {
                    surv = true;
                }
            }
            if (surv) a.rec[i].w = r.w | kRecSurvivor;
        }
        // A return whose voxel an earlier call integrated needs no eq. 4
        // window: that return stamped the same masks over the same window
        // (the masks depend on the offset only), and AND only lowers them. Its
        // voxel reads mask 0 (n = 0 only at distance 0; dedup keeps one
        // return per voxel in a scan, so this call has not written it). The
        // apply kernels then skip the window (bit 15 of the record word,
        // free when the kernel set has at most 32768 bins).
        uint32_t revisit = 0u;
        if (surv && a.revisit_ok) {
            const DevGrid &g = a.grids[a.scans[s].grid];
            if (g.revisit_skip) {
                const size_t v = (size_t)r.x + (size_t)g.nx * ((size_t)r.y + (size_t)g.ny * (size_t)r.z);
                revisit = glob(g.mask)[v] == 0u ? kRecRevisit : 0u;
            }
        }
        uint32_t c[SC_N];
        c[SC_INVALID] = st == kStInvalid;
        c[SC_OOB] = st == kStOob;
        c[SC_DUP] = st == kStOk && !surv;
        c[SC_INT] = surv;
        c[SC_SHADOW] = surv ? a.tab.sh_start[(r.w & 0xFFFFu) + 1] - a.tab.sh_start[r.w & 0xFFFFu] : 0u;
        c[SC_REVISIT] = revisit != 0u;
        // statistics: one atomic per counter per workgroup when all of its
        // points are in one scan, else one per scan per wavefront
        const uint32_t last = min(n, base + blockDim.x) - 1u;
        const uint32_t s_lo = find_scan(a.scans, info->n_scans, base);
        if (s_lo == find_scan(a.scans, info->n_scans, last)) {
#pragma unroll
            for (int f = 0; f < SC_N; ++f) {
                const uint32_t v = wave_sum_u32(c[f]);
                if (lane() == 0) s_red[f][threadIdx.x >> 6] = v;
            }
        } else {
#pragma unroll
            for (int f = 0; f < SC_N; ++f) wave_add(a.scan_ctr, s, (uint32_t)f, c[f]);
        }
        uint32_t tot;
        const uint32_t pos = block_excl_scan<kSelThreads>(surv ? 1u : 0u, s_tmp, tot);  // syncs s_red too
        if (s_lo == find_scan(a.scans, info->n_scans, last) && threadIdx.x < SC_N) {
            unsigned long long sum = 0;
            for (int k = 0; k < kSelThreads / 64; ++k) sum += s_red[threadIdx.x][k];
            if (sum) atomicAdd(&a.scan_ctr[(size_t)s_lo * SC_N + threadIdx.x], sum);
        }
        if (tot) {
            if (threadIdx.x == 0) s_base = atomicAdd(&a.ctrl->n_survivors, tot);
            __syncthreads();
            // the record word carries the bin (bits 0-15) and the grid (bits
            // 16-31; calls of more grids take the brick strategy)
            if (surv)
                a.surv_rec[s_base + pos] =
                    make_uint4(r.x, r.y, r.z, (r.w & 0xFFFFu) | revisit | (a.scans[s].grid << 16));
        }
        __syncthreads();  // s_red and s_base are reused by the next round
    }
    // The statistics go out from the apply pass (its workgroup 0), which
    // starts after this pass has finished (see stats_out).
}

// One wavefront per surviving point, straight into HBM (any kernel size,
// binning and grid): read-first atomicAnd (eq. 4) and the guard-bit counter
// (eqs. 5-6): every add that sees a raw count >= H_max is cancelled, and the
// add that sees T - 1 clears the sign. Bits 16-30 absorb the transient
// overshoot of concurrent adds. The lanes cover floor(64 / K) rows of K cells
// per pass; each lane issues the loads of kAtomicBatch passes before it
// compares any of them, and the shadow adds of a point go out together.
constexpr int kAtomicBatch = 8;
constexpr int kShadowBatch = 4;
constexpr uint32_t kXcds = 8;           // accelerator complex dies of the MI355X

__global__ __launch_bounds__(kPtThreads) void k_apply_atomic(PipeArgs a, const CallInfo *info) {
    if (blockIdx.x == 0) stats_out(a, info);
    __shared__ uint32_t lut[kLutMax];
    const DevTables &t = a.tab;
    for (uint32_t q = threadIdx.x; q < t.n_q; q += blockDim.x) lut[q] = t.mask_by_q[q];
    __syncthreads();
    const int K = t.K, R = t.R;
    const bool l1 = t.metric == DBTSDF_DIST_L1;
    // XCD-aware split of the survivor list, as in k_apply_points
    const uint32_t n_all = a.ctrl->n_survivors;
    const uint32_t n_xcd = (gridDim.x % kXcds) == 0 ? kXcds : 1u;
    const uint32_t xcd = blockIdx.x % n_xcd, slot = blockIdx.x / n_xcd;
    const uint32_t lo = (uint32_t)((uint64_t)n_all * xcd / n_xcd);
    const uint32_t n_surv = (uint32_t)((uint64_t)n_all * (xcd + 1) / n_xcd);
    const uint32_t waves = (gridDim.x / n_xcd) * (blockDim.x >> 6);
    const uint32_t l = lane();
    const uint32_t wx = (uint32_t)K, rpi = 64u / wx, xi = l % wx, ri = l / wx;
    const bool lane_on = ri < rpi;
    const uint32_t rows = (uint32_t)(K * K);
    const uint32_t mag = ((1u << 20) + wx - 1u) / wx;
    const int ox = (int)xi - R;
    for (uint32_t e = lo + slot * (blockDim.x >> 6) + (threadIdx.x >> 6); e < n_surv; e += waves) {
        const uint4 r = a.surv_rec[e];
        const DevGrid g = uniform_grid(a.grids[r.w >> 16]);
        const bool revisit = a.revisit_ok && (r.w & kRecRevisit);
        // the window's first cell (x - R, y - R, z - R); the front end admitted
        // only points whose whole window lies in the grid
        const size_t corner = (size_t)(r.x - (uint32_t)R) +
                              (size_t)g.nx * ((size_t)(r.y - (uint32_t)R) + (size_t)g.ny * (size_t)(r.z - (uint32_t)R));
        gu32 *mb = glob(g.mask) + corner;
        gu32 *pb = glob(g.packed) + corner;
        // (a return whose voxel an earlier call integrated skips its window)
        for (uint32_t r0 = 0; !revisit && r0 < rows; r0 += rpi * kAtomicBatch) {
            uint32_t old[kAtomicBatch], m[kAtomicBatch];
            size_t off[kAtomicBatch];
            bool on[kAtomicBatch];
#pragma unroll
            for (int u = 0; u < kAtomicBatch; ++u) {
                const uint32_t rr = r0 + (uint32_t)u * rpi + ri;
                on[u] = lane_on && rr < rows;
                const uint32_t rz = (rr * mag) >> 20;
                const uint32_t ry = rr - rz * wx;
                const int oy = (int)ry - R, oz = (int)rz - R;
                const uint32_t q = l1 ? (uint32_t)(abs(ox) + abs(oy) + abs(oz)) : (uint32_t)(ox * ox + oy * oy + oz * oz);
                m[u] = on[u] ? lut[q] : 0xFFFFFFFFu;
                off[u] = (size_t)xi + (size_t)g.nx * ((size_t)ry + (size_t)g.ny * (size_t)rz);
                old[u] = on[u] ? mb[off[u]] : 0u;
            }
#pragma unroll
            for (int u = 0; u < kAtomicBatch; ++u)
                if (on[u] && (old[u] & m[u]) != old[u]) g_and(mb + off[u], m[u]);
        }
        const uint32_t bin = r.w & (a.revisit_ok ? kRowBinMask : 0xFFFFu);
        const uint32_t s0 = t.sh_start[bin], s1 = t.sh_start[bin + 1];
        for (uint32_t j0 = s0; j0 < s1; j0 += 64u * kShadowBatch) {
            uint32_t ov[kShadowBatch];
            size_t so[kShadowBatch];
            bool son[kShadowBatch];
#pragma unroll
            for (int k = 0; k < kShadowBatch; ++k) {
                const uint32_t j = j0 + l + 64u * (uint32_t)k;
                son[k] = j < s1;
                const uint32_t pk = son[k] ? t.sh_off[j] : 0u;
                so[k] = (size_t)(pk & 255u) + (size_t)g.nx * ((size_t)((pk >> 8) & 255u) + (size_t)g.ny * (size_t)((pk >> 16) & 255u));
                ov[k] = son[k] ? g_add(pb + so[k], 1u) : 0u;
            }
#pragma unroll
            for (int k = 0; k < kShadowBatch; ++k) {
                if (!son[k]) continue;
                const uint32_t raw = ov[k] & 0x7FFFFFFFu;
                if (raw >= g.hmax) g_sub(pb + so[k], 1u);
                else if (g.T >= 1u && raw == g.T - 1u) g_and(pb + so[k], 0x7FFFFFFFu);
            }
        }
    }
}

// The same per-point update, reading the window row by row in aligned
// 16-byte quads. A window row of K cells at x in [px - R, px + R] lies in at
// most four quads starting at x0 = (px - R) rounded down to a multiple of 4,
// so four lanes cover a row and a wavefront covers 16 rows per load: about
// eight vector loads per point, each lane's 16 bytes contiguous, instead of
// K^3 / 64 dword loads whose lanes scatter over six rows. (The L1 tag lookups
// of the scattered dword form bound the earlier version of this kernel.)
// Each workgroup keeps in LDS, per alignment phase of the window and row, the
// eq. 3 masks of the four cells a lane covers (16 bits each, -1 outside the
// window): one 8-byte LDS read per row. Eq. 4 is the read-first atomicAnd
// where the mask loses bits. The cube bins' shadows are offset lists in LDS;
// their counters take the guard-bit atomics of eqs. 5-6, issued together with
// the window loads so that one memory round trip serves both. The tables do
// not depend on the grid: a point's row and shadow offsets are formed from
// its grid's dimensions, and its grid index rides in its survivor record, so
// a batch of scans into many grids runs the same loop as a single scan.
// kPointsPerWave consecutive survivors (neighbours in scan order, whose
// windows overlap) go to one wave and their loads are in flight together:
// fewer waves keep the memory system as busy, over a smaller L2 working set
// of windows. Needs Nx % 4 == 0 (16-byte aligned rows).
constexpr int kQuadIters = (int)kRowPad * 4 / 64;
constexpr int kShadowIters = 2;         // at most 128 shadow cells per bin
constexpr int kPointsPerWave = 2;
constexpr uint32_t kImgQuads = kImgWords / 4;
constexpr uint32_t kImgCopies = (kImgQuads + kPtThreads - 1) / kPtThreads;

// ONE: the call holds a single scan (every point in grid 0)
template <bool ONE>
__global__ __launch_bounds__(kPtThreads) void k_apply_points(PipeArgs a, const CallInfo *info) {
    if (blockIdx.x == 0) stats_out(a, info);
    // the kernel set's tables (layout in internal.h), copied in whole: every
    // thread's 16-byte loads are in flight together
    __shared__ uint4 s_img[kImgQuads];
    const uint2(*mtab)[kRowPad] = reinterpret_cast<const uint2(*)[kRowPad]>(reinterpret_cast<uint32_t *>(s_img) + kImgMtab);
    const uint32_t *sh_pk = reinterpret_cast<const uint32_t *>(s_img) + kImgShPk;
    const uint32_t *sh_bits = reinterpret_cast<const uint32_t *>(s_img) + kImgShBits;
    const uint32_t *sh_rng = reinterpret_cast<const uint32_t *>(s_img) + kImgShRng;
    constexpr int NP = kPointsPerWave;
    const DevTables &t = a.tab;
    const int K = t.K, R = t.R, K2 = K * K;
    const uint32_t l = lane();
    static_assert(kImgQuads % kPtThreads == 0, "whole copy rounds");
#pragma unroll
    for (uint32_t c = 0; c < kImgCopies; ++c) s_img[threadIdx.x + c * kPtThreads] = t.row_image[threadIdx.x + c * kPtThreads];

    // XCD-aware split: workgroups are dealt to the eight XCDs round-robin, so
    // workgroup b runs on XCD b % 8. Each XCD takes one contiguous eighth of
    // the survivor list (points in scan order are spatial neighbours whose
    // windows overlap), so the mask words a neighbourhood shares are fetched
    // into one L2 instead of eight.
    const uint32_t n_all = a.ctrl->n_survivors;
    const uint32_t n_xcd = (gridDim.x % kXcds) == 0 ? kXcds : 1u;
    const uint32_t xcd = blockIdx.x % n_xcd, slot = blockIdx.x / n_xcd;
    const uint32_t lo = (uint32_t)((uint64_t)n_all * xcd / n_xcd);
    const uint32_t hi = (uint32_t)((uint64_t)n_all * (xcd + 1) / n_xcd);
    const uint32_t wpb = blockDim.x >> 6;
    const uint32_t waves = (gridDim.x / n_xcd) * wpb;
    const uint32_t wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __syncthreads();

    const uint32_t qd = l & 3u;      // the lane's quad within a row
    const uint32_t rsub = l >> 2;    // the lane's row within a pass of 16 rows
    // the lane's window rows: (dy, dz) of row rsub + 16 k, relative to the
    // window's first row
    uint32_t rdy[kQuadIters], rdz[kQuadIters];
#pragma unroll
    for (int k = 0; k < kQuadIters; ++k) {
        const uint32_t row = rsub + 16u * k;
        rdy[k] = row < (uint32_t)K2 ? row % (uint32_t)K : 0u;
        rdz[k] = row < (uint32_t)K2 ? row / (uint32_t)K : 0u;
    }
    const uint32_t stride = waves * (uint32_t)NP;
    const uint32_t first = lo + (slot * wpb + wid) * (uint32_t)NP;
    // the next round's records are loaded one round ahead, as vector loads
    // that complete together with this round's window loads, so a round
    // costs one memory round trip
    auto fetch = [&](uint32_t e) {
        uint32_t v = e;
        asm volatile("" : "+v"(v));  // per-lane address: a vector load, counted with the window loads
        return a.surv_rec[v];
    };
    uint4 rn[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) rn[p] = first + p < hi ? fetch(first + p) : make_uint4(0u, 0u, 0u, 0u);
    // the grid of the last point seen (loaded again only when it changes)
    uint32_t cur_gi = 0u;
    DevGrid cur_g = uniform_grid(a.grids[0]);
    for (uint32_t e = first; e < hi; e += stride) {
        uint4 r[NP];
        bool live[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            r[p] = make_uint4(__builtin_amdgcn_readfirstlane(rn[p].x), __builtin_amdgcn_readfirstlane(rn[p].y),
                              __builtin_amdgcn_readfirstlane(rn[p].z), __builtin_amdgcn_readfirstlane(rn[p].w));
            live[p] = e + p < hi;
        }
#pragma unroll
        for (int p = 0; p < NP; ++p)
            if (e + stride + p < hi) rn[p] = fetch(e + stride + p);
        DevGrid g[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if constexpr (!ONE) {
                const uint32_t gi = r[p].w >> 16;
                if (live[p] && gi != cur_gi) {
                    cur_gi = gi;
                    cur_g = uniform_grid(a.grids[gi]);
                }
            }
            g[p] = cur_g;
        }
        // every point's window loads, then every point's shadow adds
        const char __attribute__((address_space(1))) *mbase[NP];
        const char __attribute__((address_space(1))) *pbase[NP];
        uint32_t sel[NP], roff[NP][kQuadIters];
        u32x4 old[NP][kQuadIters];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            // x0: first quad of the window rows; the front end admitted only
            // points whose whole window lies in the grid, and Nx % 4 == 0 keeps
            // every quad that meets the window inside its grid row
            const uint32_t x0 = (r[p].x - (uint32_t)R) & ~3u;
            const size_t row0 = (size_t)g[p].nx * ((size_t)(r[p].y - R) + (size_t)g[p].ny * (size_t)(r[p].z - R));
            mbase[p] = reinterpret_cast<const char __attribute__((address_space(1))) *>(glob(g[p].mask) + row0 + x0);
            pbase[p] = reinterpret_cast<const char __attribute__((address_space(1))) *>(
                glob(g[p].packed) + row0 + (size_t)(r[p].x - (uint32_t)R));
            sel[p] = 4u * qd + 3u - ((r[p].x - (uint32_t)R) & 3u);
            // a return in a voxel integrated by an earlier call skips its window
            const bool qon = live[p] && !(r[p].w & kRecRevisit) && x0 + 4u * qd <= r[p].x + (uint32_t)R;
            const uint32_t sy = 4u * g[p].nx, sz = 4u * g[p].nx * g[p].ny;  // row strides in bytes
#pragma unroll
            for (int k = 0; k < kQuadIters; ++k) {
                roff[p][k] = rdy[k] * sy + rdz[k] * sz;   // 32 bits: the call checked 8 R (1 + Nx + Nx Ny) < 2^32
                const bool on = qon && (int)(rsub + 16u * k) < K2;
                old[p][k] = on ? *reinterpret_cast<gu32x4 *>(mbase[p] + roff[p][k] + 16u * qd)
                               : u32x4{0u, 0u, 0u, 0u};
            }
        }
        // shadow counters (eq. 5). A cell in the shadows of several points of
        // the round (same grid) takes one add of their number, issued by the
        // first of them; the others skip it
        uint32_t ov[NP][kShadowIters], soff[NP][kShadowIters], cnt[NP][kShadowIters];
        bool son[NP][kShadowIters];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const uint32_t bin = r[p].w & kRowBinMask;
            const uint32_t s0 = sh_rng[bin], s1 = live[p] ? sh_rng[bin + 1] : s0;
#pragma unroll
            for (int k = 0; k < kShadowIters; ++k) {
                const uint32_t j = s0 + l + 64u * k;
                son[p][k] = j < s1;
                const uint32_t pk = son[p][k] ? sh_pk[j] : 0u;
                uint32_t c = 1u;
#pragma unroll
                for (int q = 0; q < NP; ++q) {
                    if (q == p || !live[q] || (!ONE && (r[q].w >> 16) != (r[p].w >> 16))) continue;
                    // the cell relative to point q, in [-3, 3]^3 when it can be in q's shadow
                    const int rx = (int)(pk & 255u) - R + (int)r[p].x - (int)r[q].x;
                    const int ry = (int)((pk >> 8) & 255u) - R + (int)r[p].y - (int)r[q].y;
                    const int rz = (int)((pk >> 16) & 255u) - R + (int)r[p].z - (int)r[q].z;
                    bool in = rx >= -3 && rx <= 3 && ry >= -3 && ry <= 3 && rz >= -3 && rz <= 3;
                    if (in) {
                        const uint32_t idx = (uint32_t)((rx + 3) + 7 * (ry + 3) + 49 * (rz + 3));
                        in = ((sh_bits[(r[q].w & kRowBinMask) * kShadowSetWords + idx / 32u] >> (idx % 32u)) & 1u) != 0u;
                    }
                    if (q < p) son[p][k] = son[p][k] && !in;
                    else c += in ? 1u : 0u;
                }
                cnt[p][k] = c;
                soff[p][k] = 4u * ((pk & 255u) + g[p].nx * (((pk >> 8) & 255u) + g[p].ny * ((pk >> 16) & 255u)));
                ov[p][k] = 0u;
                if (son[p][k]) ov[p][k] = g_add((gu32 *)(pbase[p] + soff[p][k]), c);
            }
        }
        // eq. 4: stored and stamped masks are both 2^n - 1, so the AND loses
        // bits exactly when old > m; every compare comes first, then the
        // atomics of a point that needs them go out in one burst (a register
        // read by an atomic in flight is not overwritten before the round ends)
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            auto masks = [&](int k, uint32_t m[4]) {
                const uint2 v = mtab[sel[p]][rsub + 16u * k];
                m[0] = (uint32_t)((int32_t)(v.x << 16) >> 16);
                m[1] = (uint32_t)((int32_t)v.x >> 16);
                m[2] = (uint32_t)((int32_t)(v.y << 16) >> 16);
                m[3] = (uint32_t)((int32_t)v.y >> 16);
            };
            // a point that loaded no window (past the end, or a revisit) has
            // nothing to compare
            if (!live[p] || (r[p].w & kRecRevisit)) continue;
            bool need = false;
#pragma unroll
            for (int k = 0; k < kQuadIters; ++k) {
                uint32_t m[4];
                masks(k, m);
                need |= (old[p][k][0] > m[0]) | (old[p][k][1] > m[1]) | (old[p][k][2] > m[2]) | (old[p][k][3] > m[3]);
            }
            if (need) {  // rare once the map has formed: the compares are redone here
#pragma unroll
                for (int k = 0; k < kQuadIters; ++k) {
                    uint32_t m[4];
                    masks(k, m);
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (old[p][k][j] > m[j]) g_and((gu32 *)(mbase[p] + (roff[p][k] + 16u * qd + 4u * j)), m[j]);
                }
            }
        }
        // eqs. 5-6 with the returns of the adds of c: an add that saw a raw
        // count >= H_max is cancelled, one that crossed H_max gives back its
        // excess, the add whose range [raw, min(raw + c, H_max)] steps over
        // T - 1 -> T clears the sign (bits 16-30 absorb the transient
        // overshoot; c = 1 is the unit scheme)
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int k = 0; k < kShadowIters; ++k) {
                // an opaque use: the returned value is not touched (and waited
                // for) before the window compares above have been issued
                asm volatile("" : "+v"(ov[p][k]));
                if (!son[p][k]) continue;
                gu32 *w = (gu32 *)(pbase[p] + soff[p][k]);
                const uint32_t raw = ov[p][k] & 0x7FFFFFFFu, c = cnt[p][k], H = g[p].hmax, T = g[p].T;
                if (raw >= H) {
                    g_sub(w, c);
                } else {
                    if (raw + c > H) g_sub(w, raw + c - H);
                    if (T >= 1u && raw < T && T <= min(raw + c, H)) g_and(w, 0x7FFFFFFFu);
                }
            }
        }
    }
}

// ======================================================== tile strategy ===
// Returns are listed by grid tile (kTileX x kTileY x kTileZ words) in the
// front pass; k_offsets lays the lists out; k_select_fill takes the survivor
// test and writes each return into its lists (a return that lost the
// first-return test leaves a hole); k_apply_tile gives each tile to one
// workgroup, which takes in LDS, per word of the tile, the smallest eq. 3
// metric value q over the windows of the tile's listed returns (ds_min; the
// mask of the smallest q is the AND of all their masks, eq. 3 being
// monotone in q) and the number of shadow hits, then reads, updates and
// writes each touched word of both planes once with plain 16-byte loads and
// stores. Every word has one owner tile, so no atomic touches the planes.

// Survivor test, statistics and list fill of the tile strategy (one thread
// per return). Only the slot's winner releases a dedup slot (as in
// k_select_atomic). The apply pass writes the statistics into the ring slot;
// workgroup 0 clears the work-item counter the next call's front pass counts
// on (every reader of it, the offsets pass, is done).
__global__ __launch_bounds__(kSelThreads) void k_select_fill(PipeArgs a, const CallInfo *info) {
    __shared__ uint32_t s_red[SC_N][kSelThreads / 64];
    const uint32_t n = info->n_points;
    const int R = a.tab.R;
    const int rs = shadow_extent(a.tab);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctrl->n_active = 0u;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        const bool live = i < n;
        uint4 r = make_uint4(0u, 0u, 0u, 0u);
        uint32_t s = 0, st = 3u;
        bool surv = false, rv = false;
        if (live) {
            r = a.rec[i];
            st = (r.w >> 16) & 3u;
            s = find_scan(a.scans, info->n_scans, i);
            if (st == kStOk) {
                if (a.scans[s].dedup) {
                    const uint32_t slot = a.pslot[i];
                    surv = a.hvals[slot] == i;
                    if (surv) {
                        a.hkeys[slot] = kHashEmpty;
                        a.hvals[slot] = 0xFFFFFFFFu;
                    }
                } else {
                    surv = true;
                }
                rv = (r.w & kRecTileRevisit) != 0u;
                const DevGrid &g = a.grids[a.scans[s].grid];
                const TileSpan sp = tile_span(r.x, r.y, r.z, rv ? rs : R);
                const uint32_t np = sp.nx * sp.ny * sp.nz;
                const uint4 e = surv ? make_uint4(r.x, r.y, r.z, (r.w & 0xFFFFu) | (rv ? kRecRevisit : 0u))
                                     : make_uint4(kTileHole, kTileHole, kTileHole, kTileHole);
                for (uint32_t j0 = 0; j0 < np; j0 += kSelUnroll) {
                    uint32_t slot[kSelUnroll], rk[kSelUnroll];
#pragma unroll
                    for (int u = 0; u < kSelUnroll; ++u) {  // independent loads, all in flight
                        const bool v = j0 + u < np;
                        slot[u] = v ? glob(g.brick_slot)[tile_ctr(g, span_tile(sp, j0 + u, g))] : 0u;
                        rk[u] = v ? a.rank[(size_t)(j0 + u) * n + i] : 0u;   // as the front pass stores them
                    }
#pragma unroll
                    for (int u = 0; u < kSelUnroll; ++u)
                        if (j0 + u < np) a.entries[slot[u] + rk[u]] = e;
                }
            }
        }
        uint32_t c[SC_N];
        c[SC_INVALID] = st == kStInvalid;
        c[SC_OOB] = st == kStOob;
        c[SC_DUP] = st == kStOk && !surv;
        c[SC_INT] = surv;
        c[SC_SHADOW] = surv ? a.tab.sh_start[(r.w & 0xFFFFu) + 1] - a.tab.sh_start[r.w & 0xFFFFu] : 0u;
        c[SC_REVISIT] = surv && rv;
        const uint32_t last = min(n, base + blockDim.x) - 1u;
        const uint32_t s_lo = find_scan(a.scans, info->n_scans, base);
        const bool one_scan = s_lo == find_scan(a.scans, info->n_scans, last);
        if (one_scan) {
#pragma unroll
            for (int f = 0; f < SC_N; ++f) {
                const uint32_t v = wave_sum_u32(c[f]);
                if (lane() == 0) s_red[f][threadIdx.x >> 6] = v;
            }
            __syncthreads();
            if (threadIdx.x < SC_N) {
                unsigned long long sum = 0;
                for (int k = 0; k < kSelThreads / 64; ++k) sum += s_red[threadIdx.x][k];
                if (sum) atomicAdd(&a.scan_ctr[(size_t)s_lo * SC_N + threadIdx.x], sum);
            }
            __syncthreads();
        } else {
#pragma unroll
            for (int f = 0; f < SC_N; ++f) wave_add(a.scan_ctr, s, (uint32_t)f, c[f]);
        }
    }
    // The statistics go out from the apply pass (its workgroup 0), which the
    // stream starts after this pass has finished: a last-workgroup count here
    // would put one returning atomic per workgroup on one address, and those
    // queue behind each other at the coherence point.
}

// One workgroup per tile work item (persistent: items dealt round-robin over
// the workgroups). LDS holds, per word of the tile, the eq. 3 stamp as a
// 16-bit mask (2^n - 1; 0xFFFF where no window reaches, the identity of the
// AND), four words to a 64-bit quad, and the shadow hit count as a byte, four
// to a 32-bit word. Each LDS row carries halo cells on both sides of the
// tile's 32 (written to, never merged, never cleared), wide enough for every
// window and shadow row of a listed return, so that a row's writes need no
// bounds test. The tile's list is taken in rounds of at most 255 entries (a
// count byte cannot overflow: an entry adds at most one hit to a word):
//   1. one thread per entry: the rows it walks, clipped to the tile in y and
//      z (the window's (y, z) rows for a return that applies its window, the
//      shadow ball's for one whose voxel an earlier call integrated), its
//      first row's stamp quad and count word, and one scan of the row counts
//      over the round, with a bitmap of the rows where an entry starts;
//   2. the rows of all entries are dealt to the lanes, 64 consecutive rows a
//      wavefront: a lane finds its entry by counting the starts below its row
//      in the bitmap, ANDs its window row's masks in with four ds_and_b64 (the
//      masks of the row kernel's table for the window's alignment phase, by
//      |dy| and |dz|: eq. 3 is even in both), and, where the row lies in the
//      shadow ball, adds the row's hits (bits of the bin's shadow row) with
//      two 64-bit adds, each on an 8-word pair of count words;
//   3. the round is merged, four 16-byte quads per thread: the stamps and
//      counts go to registers (their LDS words reset for the next round), the
//      loads of the words they touch are issued together, then (one wait)
//      mask &= the stamp (stored when changed); h = min(h + c, H_max) with the
//      sign cleared on the crossing h < T <= h + c (eqs. 5-6 for c unit
//      steps). A tile of several rounds merges each in turn (AND is idempotent
//      and c then d steps are c + d steps).
// Needs the row kernel's tables (K <= 11, at most 31 bins, r_s^2 <= 9).
constexpr int kTileThreads = 256;
constexpr uint32_t kTileRound = 255;                    // entries per round
constexpr uint32_t kTileRows = kTileY * kTileZ;         // (y, z) rows of a tile
constexpr uint32_t kTileQx = kTileX / 4;                // quads per row
// A window row, cells lx - R .. lx + R with lx in [-R, 31 + R], takes the four
// quads from (lx - R) >> 2, in [-3, 10]: LDS rows hold three halo quads on
// either side of the tile's eight and are padded to 15 quads (odd: lanes on
// neighbouring rows fall in different banks), z layers to 241 quads.
constexpr uint32_t kHaloQ = 3;
constexpr uint32_t kTilePq = kTileQx + 2 * kHaloQ + 1;
constexpr uint32_t kTileLayer = kTilePq * kTileY + 1;
constexpr uint32_t kTileSlots = kTileLayer * kTileZ;
// The hit counts: a shadow row, cells lx - 3 .. lx + 3, adds to the two 8-cell
// pairs of count words from (lx - 3) >> 3, in [-1, 5]: rows hold one halo pair
// before the tile's four and two after (14 words), z layers padded to 226.
constexpr uint32_t kHaloC = 2;   // count words before the tile's first
constexpr uint32_t kCntPitch = kTileQx + 3u * 2u, kCntLayer = kCntPitch * kTileY + 2, kCntSlots = kCntLayer * kTileZ;
constexpr uint32_t kTileQuadsPerThread = kTileRows * kTileQx / kTileThreads;
constexpr uint32_t kShadowRows = 49;                    // (dy, dz) in [-3, 3]^2
constexpr uint32_t kRowsMax = kTileRound * 11u * kTileZ;   // rows of a round (windows of 11 rows, clipped z)
constexpr uint32_t kRowBlocks = (kRowsMax + 63) / 64;
constexpr uint32_t kMtRows = 6u * 6u;                   // window rows by (|dy|, |dz|), K <= 11
static_assert(kTileRows * kTileQx % kTileThreads == 0, "whole quads per thread");
static_assert(kTileRound < kTileThreads, "one entry per thread in the set-up");
static_assert(kTileLayer * (kTileZ - 1) + kTilePq * (kTileY - 1) + 2 * kHaloQ + kTileQx - 1 < kTileSlots &&
                  kCntLayer * (kTileZ - 1) + kCntPitch * (kTileY - 1) + kCntPitch - 1 < kCntSlots &&
                  kTileSlots < 2048 && kCntSlots < 2048, "row bases fit 11 bits");
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

// Division of a 32-bit n by a divisor d >= 1 fixed for many divisions, as a
// multiply-high and shifts (Granlund and Montgomery's round-up method with a
// 33-bit multiplier: l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1,
// t = mulhi(m, n), n / d = (t + ((n - t) >> 1)) >> (l - 1); for d = 1 the
// shifts are 0 and t = 0). Exact for every n and d.
struct FastDiv {
    uint32_t m, s1, s2;
};
__device__ __forceinline__ FastDiv fastdiv_of(uint32_t d) {
    const uint32_t l = d > 1u ? 32u - (uint32_t)__clz(d - 1u) : 0u;
    const uint64_t m = ((((uint64_t)1 << l) - d) << 32) / d + 1u;
    // (d is uniform where this is used: the fields go to scalar registers)
    return FastDiv{(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)m), l ? 1u : 0u,
                   (uint32_t)__builtin_amdgcn_readfirstlane(l ? l - 1u : 0u)};
}
__device__ __forceinline__ uint32_t fastdiv(uint32_t n, const FastDiv &f) {
    const uint32_t t = __umulhi(n, f.m);
    return (t + ((n - t) >> f.s1)) >> f.s2;
}

__device__ __forceinline__ uint32_t spread4(uint32_t b4) {   // bit j -> byte j
    return (b4 * 0x00204081u) & 0x01010101u;
}

__global__ __launch_bounds__(kTileThreads, 4) void k_apply_tile(PipeArgs a) {
    if (blockIdx.x == 0) stats_out(a, reinterpret_cast<const CallInfo *>(a.ctrl + 1));
    __shared__ __align__(16) uint2 stamp[kTileSlots];      // 4 x 16-bit masks per quad
    __shared__ __align__(16) uint32_t cnt[kCntSlots];      // 4 x 8-bit hit counts per word of counts
    // masks by (phase, |dy| + 6 |dz|, quad)
    __shared__ __align__(16) unsigned long long mt[4][kMtRows][4];
    __shared__ uint8_t smask[kRowBins * kShadowRows];               // shadow x bits (dx + 3) per (bin, dy, dz)
    // per entry with rows, in round order: box and point (tile-local), row
    // magic and bin, first row
    __shared__ uint4 info[kTileRound];
    __shared__ unsigned long long starts[kRowBlocks];  // bit: an entry's first row
    __shared__ uint16_t block_base[kRowBlocks];        // entries with rows starting before the block
    __shared__ uint32_t s_scan[kTileThreads / 64 + 1];
    __shared__ uint32_t s_magic[kTileY + 1];
    const DevTables &t = a.tab;
    if (threadIdx.x <= kTileY) s_magic[threadIdx.x] = threadIdx.x ? (65536u + threadIdx.x - 1u) / threadIdx.x : 0u;
    const int R = t.R, K = t.K;
    const int rs = shadow_extent(t);
    {
        // the row kernel's table mtab[sel][row] (sel = 4 qd + 3 - phase, row
        // (dy + R) + K (dz + R)) for dy, dz >= 0, laid out by (phase, row) so
        // that a row's four quads are contiguous
        const uint2 *mtab = reinterpret_cast<const uint2 *>(t.row_image) + kImgMtab / 2;
        for (uint32_t i = threadIdx.x; i < 4u * kMtRows * 4u; i += kTileThreads) {
            const uint32_t ph = i / (kMtRows * 4u), row = (i / 4u) % kMtRows, qd = i % 4u;
            const int ady = (int)(row % 6u), adz = (int)(row / 6u);
            const uint2 m = ady <= R && adz <= R ? mtab[(4u * qd + 3u - ph) * kRowPad + (uint32_t)(ady + R + K * (adz + R))]
                                                 : make_uint2(~0u, ~0u);
            mt[ph][row][qd] = (unsigned long long)m.x | ((unsigned long long)m.y << 32);
        }
        // stamps and counts start at the identity; the merge resets the
        // words it reads (the halo cells are never read)
        for (uint32_t q = threadIdx.x; q < kTileSlots; q += kTileThreads) stamp[q] = make_uint2(~0u, ~0u);
        for (uint32_t q = threadIdx.x; q < kCntSlots; q += kTileThreads) cnt[q] = 0u;
        // each bin's shadow set as 7-bit x rows, from its 343-bit set (bits
        // (dx + 3) + 7 (dy + 3) + 49 (dz + 3))
        const uint32_t *bits = reinterpret_cast<const uint32_t *>(t.row_image) + kImgShBits;
        for (uint32_t i = threadIdx.x; i < t.n_bins * kShadowRows; i += kTileThreads) {
            const uint32_t b = i / kShadowRows, p = 7u * (i % kShadowRows);
            const uint32_t w = p >> 5, o = p & 31u;
            uint32_t v = bits[b * kShadowSetWords + w] >> o;
            if (o > 25u) v |= bits[b * kShadowSetWords + w + 1] << (32u - o);
            smask[i] = (uint8_t)(v & 0x7Fu);
        }
    }
    const uint32_t l = lane();
    const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr uint32_t kWaves = kTileThreads / 64;
    const uint32_t n_work = a.ctrl->n_work;
    // Work items are dealt round-robin. The next item's descriptor and first
    // round of entries (a thread holds at most one of them) are loaded one
    // item ahead, the descriptor of the item after it two ahead. A wait for a
    // vector load also waits for every vector load and store issued before it
    // (they complete in order), so each is taken into registers where that
    // costs nothing: the entries before the plane loads of a round are
    // issued, the descriptor with those plane loads (it is loaded right after
    // them); no wait comes right after a merge's stores, and every barrier
    // here orders LDS only.
    const uint32_t G = gridDim.x;
    // Loads of a work item's descriptor (uniform, but loaded per lane so that
    // it is waited for with the vector loads) and of one entry per lane; zero
    // where the condition fails. Both go to global memory directly.
    auto vload = [&](const uint4 *p, uint32_t i, bool c) {
        uint32_t v = i;
        asm volatile("" : "+v"(v));
        uint4 r = make_uint4(0u, 0u, 0u, 0u);
        if (c) r = gload4(p, v);
        return r;
    };
    auto eload = [&](uint32_t i, bool c) {
        uint4 r = make_uint4(0u, 0u, 0u, 0u);
        if (c) r = gload4(a.entries, i);
        return r;
    };
    uint32_t wi = blockIdx.x;
    uint4 wk = vload(a.work, wi, wi < n_work);
    uint4 ent_cur = eload(wk.z + threadIdx.x, wi < n_work && threadIdx.x < min(wk.w & 0x7FFFFFFFu, kTileRound));
    uint4 wk_next = vload(a.work, wi + G, wi + G < n_work);
    uint4 wk_nn = make_uint4(0u, 0u, 0u, 0u);   // the descriptor of the item after next
    for (uint32_t c = threadIdx.x; c < kRowBlocks; c += kTileThreads) starts[c] = 0ull;
    // the grid of the last item (loaded again only when it changes), and its
    // tile counts per row and layer as divisors
    uint32_t cur_gi = 0u;
    DevGrid g = uniform_grid(a.grids[0]);
    g.nbx = __builtin_amdgcn_readfirstlane(g.nbx);
    g.nby = __builtin_amdgcn_readfirstlane(g.nby);
    FastDiv div_x = fastdiv_of(g.nbx), div_y = fastdiv_of(g.nby);
    // The merge of a round: each thread takes the stamps and counts of its
    // quads into registers and issues the loads of the words they touch
    // (issue), then updates and stores them (finish). Other workgroups on the
    // CU cover the loads' latency.
    uint2 sq[kTileQuadsPerThread];
    uint32_t cq[kTileQuadsPerThread];
    u32x4 om[kTileQuadsPerThread], op[kTileQuadsPerThread];
    // A thread's quads: x 4 (tid mod 8), y (tid / 8) mod 16 and z tid / 128
    // + kQz k for its k-th; the same in every tile.
    constexpr uint32_t kQz = kTileThreads / (kTileQx * kTileY);
    static_assert(kTileThreads % (kTileQx * kTileY) == 0 && kQz * kTileQuadsPerThread == kTileZ, "quads per thread");
    const uint32_t q_x = 4u * (threadIdx.x % kTileQx), q_y = (threadIdx.x / kTileQx) % kTileY,
                   q_z = threadIdx.x / (kTileQx * kTileY);
    const uint32_t s_off = kHaloQ + q_x / 4u + kTilePq * q_y + kTileLayer * q_z;   // stamp slot of quad 0 (+ kTileLayer kQz k)
    const uint32_t c_off = kHaloC + q_x / 4u + kCntPitch * q_y + kCntLayer * q_z;  // count slot of quad 0 (+ kCntLayer kQz k)
    // the merge: grid, first word, word step between quads, the quad's cells
    // and which quads lie inside the grid with 16-byte aligned rows
    DevGrid pg = g;
    size_t plin = 0, pstep = 0;
    uint32_t pgx = 0, pgy = 0, pgz = 0;
    bool pxy = false;
    auto issue = [&](int X0, int Y0, int Z0, const DevGrid &gi) {
        pg = gi;
        pgx = (uint32_t)X0 + q_x;
        pgy = (uint32_t)Y0 + q_y;
        pgz = (uint32_t)Z0 + q_z;
        plin = (size_t)pgx + (size_t)gi.nx * ((size_t)pgy + (size_t)gi.ny * (size_t)pgz);
        pstep = (size_t)kQz * (size_t)gi.nx * (size_t)gi.ny;
        pxy = (gi.nx & 3u) == 0u && pgx + 3u < gi.nx && pgy < gi.ny;
#pragma unroll
        for (uint32_t k = 0; k < kTileQuadsPerThread; ++k) {
            sq[k] = stamp[s_off + kTileLayer * kQz * k];
            cq[k] = cnt[c_off + kCntLayer * kQz * k];
            stamp[s_off + kTileLayer * kQz * k] = make_uint2(~0u, ~0u);
            cnt[c_off + kCntLayer * kQz * k] = 0u;
            if (pxy && pgz + kQz * k < gi.nz) {
                const size_t lin = plin + (size_t)k * pstep;
                if ((sq[k].x & sq[k].y) != ~0u) om[k] = *reinterpret_cast<const gu32x4 *>(glob(gi.mask) + lin);
                if (cq[k] != 0u) op[k] = *reinterpret_cast<const gu32x4 *>(glob(gi.packed) + lin);
            }
        }
    };
    auto finish = [&]() {
        // All the loaded words taken into registers first: one wait for the
        // loads, issued a round ago. (Vector stores count against the same
        // counter, so a wait between this thread's stores would also wait
        // for the stores before it.)
#pragma unroll
        for (uint32_t k = 0; k < kTileQuadsPerThread; ++k) asm volatile("" : "+v"(om[k]), "+v"(op[k]));
        asm volatile("" : "+v"(wk_nn.x), "+v"(wk_nn.y), "+v"(wk_nn.z), "+v"(wk_nn.w));
#pragma unroll
        for (uint32_t k = 0; k < kTileQuadsPerThread; ++k) {
            const bool nm = (sq[k].x & sq[k].y) != ~0u, nh = cq[k] != 0u;
            if (!nm && !nh) continue;
            // the 16-bit stamps sign-extended: the identity 0xFFFF becomes
            // ~0, and every eq. 3 mask (below 2^15) stays as it is
            const uint32_t mm[4] = {(uint32_t)(int32_t)(int16_t)(sq[k].x & 0xFFFFu), (uint32_t)((int32_t)sq[k].x >> 16),
                                    (uint32_t)(int32_t)(int16_t)(sq[k].y & 0xFFFFu), (uint32_t)((int32_t)sq[k].y >> 16)};
            const uint32_t gz = pgz + kQz * k;
            const size_t lin = plin + (size_t)k * pstep;
            if (pxy && gz < pg.nz) {
                if (nm) {
                    const uint32_t o[4] = {om[k][0], om[k][1], om[k][2], om[k][3]};
                    uint32_t nw[4];
                    bool ch = false;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        nw[j] = o[j] & mm[j];
                        ch |= nw[j] != o[j];
                    }
                    if (ch) gstore4(pg.mask + lin, nw[0], nw[1], nw[2], nw[3]);
                }
                if (nh) {
                    // (a word without hits comes out unchanged: its bits 16-30
                    // are clear and its counter is at most H_max, invariants
                    // of the planes)
                    const uint32_t o[4] = {op[k][0], op[k][1], op[k][2], op[k][3]};
                    uint32_t nw[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const uint32_t c = (cq[k] >> (8 * j)) & 0xFFu;
                        const uint32_t h0 = o[j] & 0xFFFFu;
                        const uint32_t h1 = min(h0 + c, pg.hmax);
                        const uint32_t sign = (h0 < pg.T && h1 >= pg.T) ? 0u : (o[j] & 0x80000000u);
                        nw[j] = sign | h1;
                    }
                    gstore4(pg.packed + lin, nw[0], nw[1], nw[2], nw[3]);
                }
                continue;
            }
            // a quad at the grid's edge, or rows not 16-byte aligned: word by word
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (pgx + (uint32_t)j >= pg.nx || pgy >= pg.ny || gz >= pg.nz) continue;
                const size_t li = lin + (size_t)j;
                if (mm[j] != ~0u) {
                    gu32 *pm = glob(pg.mask) + li;
                    const uint32_t old = *pm;
                    const uint32_t nw = old & mm[j];
                    if (nw != old) *pm = nw;
                }
                const uint32_t c = (cq[k] >> (8 * j)) & 0xFFu;
                if (c) {
                    gu32 *pp = glob(pg.packed) + li;
                    const uint32_t old = *pp;
                    const uint32_t h0 = old & 0xFFFFu;
                    const uint32_t h1 = min(h0 + c, pg.hmax);
                    const uint32_t sign = (h0 < pg.T && h1 >= pg.T) ? 0u : (old & 0x80000000u);
                    *pp = sign | h1;
                }
            }
        }
    };
    while (wi < n_work) {
        // the item's descriptor, uniform: into scalar registers
        const uint32_t brick = __builtin_amdgcn_readfirstlane(wk.x), gi = __builtin_amdgcn_readfirstlane(wk.y);
        const uint32_t first = __builtin_amdgcn_readfirstlane(wk.z);
        const uint32_t total = __builtin_amdgcn_readfirstlane(wk.w) & 0x7FFFFFFFu;
        if (gi != cur_gi) {
            cur_gi = gi;
            g = uniform_grid(a.grids[cur_gi]);
            g.nbx = __builtin_amdgcn_readfirstlane(g.nbx);   // (waited for here, not at every item)
            g.nby = __builtin_amdgcn_readfirstlane(g.nby);
            div_x = fastdiv_of(g.nbx);
            div_y = fastdiv_of(g.nby);
        }
        const uint32_t bq = fastdiv(brick, div_x), tz = fastdiv(bq, div_y);
        const uint32_t tx = brick - bq * g.nbx, ty = bq - tz * g.nby;
        const int X0 = (int)(tx * kTileX), Y0 = (int)(ty * kTileY), Z0 = (int)(tz * kTileZ);
        // the next item's first round of entries, where this item's last
        // round is its first
        const uint32_t next_first = __builtin_amdgcn_readfirstlane(wk_next.z);
        const uint32_t next_nb =
            wi + G < n_work ? min(__builtin_amdgcn_readfirstlane(wk_next.w) & 0x7FFFFFFFu, kTileRound) : 0u;
        if (total == 0u) {   // (an item without entries: waited for at once)
            ent_cur = eload(next_first + threadIdx.x, threadIdx.x < next_nb);
            wk_nn = vload(a.work, wi + 2u * G, wi + 2u * G < n_work);
            asm volatile("" : "+v"(ent_cur.x), "+v"(ent_cur.y), "+v"(ent_cur.z), "+v"(ent_cur.w), "+v"(wk_nn.x),
                              "+v"(wk_nn.y), "+v"(wk_nn.z), "+v"(wk_nn.w));
        }
        for (uint32_t b0 = 0; b0 < total; b0 += kTileRound) {
            const uint32_t nb = min(total - b0, kTileRound);
            lds_barrier();   // the previous round's (or item's) merge is done with the arrays
            const uint4 r = ent_cur;
            // the next round's entries: this item's next round, else the next item's first
            const bool more = b0 + kTileRound < total;
            const uint32_t pidx = more ? first + b0 + kTileRound : next_first;
            const uint32_t pcnt = more ? min(total - b0 - kTileRound, kTileRound) : next_nb;
            uint4 pe = eload(pidx + threadIdx.x, threadIdx.x < pcnt);
            // per entry (thread e): the rows it walks, clipped to the tile
            uint32_t rows = 0;
            uint4 inf = make_uint4(0u, 0u, 0u, 0u);
            if (threadIdx.x < nb && r.x != kTileHole) {
                const int lx = (int)r.x - X0, ly = (int)r.y - Y0, lz = (int)r.z - Z0;
                const bool rv = a.revisit_ok && (r.w & kRecRevisit);
                const uint32_t bin = r.w & (a.revisit_ok ? kRowBinMask : 0xFFFFu);
                const int ext = rv ? rs : R;
                if (ext >= 0) {
                    const int ya = max(ly - ext, 0), yb = min(ly + ext, (int)kTileY - 1);
                    const int za = max(lz - ext, 0), zb = min(lz + ext, (int)kTileZ - 1);
                    const int wy = yb - ya + 1, wz = zb - za + 1;
                    if (wy > 0 && wz > 0 && lx + ext >= 0 && lx - ext < (int)kTileX) {
                        rows = (uint32_t)(wy * wz);
                        // the first row's stamp quad (the window's quads from
                        // (lx - R) >> 2) and count word (the shadow's pairs
                        // from (lx - 3) >> 3), halo included, and its (dy, dz).
                        // info: x first row of the round (set below), y the
                        // magic of wy; z stamp quad (bits 0-10), count word
                        // (11-21), bin (22-26), revisit (27), window phase
                        // (28-29); w wy (0-3), the shadow row's shift (4-6),
                        // dy + 8 (8-11), dz + 8 (12-15)
                        const int xs = lx - R, sx = lx - 3;
                        const uint32_t qb = (uint32_t)((xs >> 2) + (int)kHaloQ) + kTilePq * (uint32_t)ya +
                                            kTileLayer * (uint32_t)za;
                        const uint32_t cb = (uint32_t)(2 * (sx >> 3) + (int)kHaloC) + kCntPitch * (uint32_t)ya +
                                            kCntLayer * (uint32_t)za;
                        inf = make_uint4(0u, s_magic[wy],   // r / wy = (r * magic) >> 16 for r < 256
                                         qb | (cb << 11) | ((bin & 31u) << 22) | (rv ? 1u << 27 : 0u) |
                                             ((uint32_t)(xs & 3) << 28),
                                         (uint32_t)wy | ((uint32_t)(sx & 7) << 4) | ((uint32_t)(ya - ly + 8) << 8) |
                                             ((uint32_t)(za - lz + 8) << 12));
                    }
                }
            }
            // one scan over the round: the rows before the entry (high bits)
            // and the entries with rows before it (low 9 bits); a round of at
            // most 64 entries has them all in wavefront 0, whose own scan
            // needs no barrier (the others take its total after the next one)
            const uint32_t sv = (rows << 9) | (rows ? 1u : 0u);
            uint32_t ex, tot;
            if (nb <= 64u) {
                const uint32_t incl = wave_incl_scan_u32(sv);
                ex = incl - sv;
                tot = __shfl(incl, 63);
                if (threadIdx.x == 63u) s_scan[kWaves] = incl;
            } else {
                ex = block_excl_scan<kTileThreads, true>(sv, s_scan, tot);
            }
            uint32_t n_rows = tot >> 9;
            uint32_t n_blocks = (n_rows + 63u) / 64u;
            if (rows) {
                const uint32_t k_e = ex & 511u, r0 = ex >> 9;
                inf.x = r0;
                info[k_e] = inf;
                atomicOr(&starts[r0 >> 6], 1ull << (r0 & 63u));
                // blocks whose first row lies after this entry's first row and
                // at or before the next one's: this entry's index + 1 entries
                // start before them
                for (uint32_t c = (r0 >> 6) + 1u; c <= min((r0 + rows) >> 6, n_blocks - 1u); ++c)
                    block_base[c] = (uint16_t)(k_e + 1u);
            }
            if (threadIdx.x == 0) block_base[0] = 0;
            lds_barrier();
            if (nb <= 64u) {
                n_rows = s_scan[kWaves] >> 9;
                n_blocks = (n_rows + 63u) / 64u;
            }
            // The rows, 64 to a wavefront, two blocks of rows at a time: the
            // look-ups of both are issued before the first write (the writes
            // are ANDs and adds, so their order does not matter). A lane's
            // entry is the last one starting at or before its row: block c's
            // entries before it plus the start bits up to the lane (block 0
            // starts with entry 0; a later block has a nonzero base); a lane
            // past the last row reads a valid entry and writes nothing.
            for (uint32_t c0 = w; c0 < n_blocks; c0 += 2u * kWaves) {
                bool win[2], sh[2];
                uint32_t qa[2], ca[2], m7[2], shf[2], bb[2];
                u64x2 m01[2], m23[2];
                unsigned long long seg[2];
                uint4 ine[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const uint32_t c = min(c0 + (uint32_t)u * kWaves, n_blocks - 1u);
                    seg[u] = starts[c];
                    bb[u] = block_base[c];
                }
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    ine[u] = info[bb[u] + (uint32_t)__popcll(seg[u] & ((2ull << l) - 1ull)) - 1u];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const uint32_t rho = 64u * (c0 + (uint32_t)u * kWaves) + l;
                    const bool on = rho < n_rows;
                    const uint4 in = ine[u];
                    const uint32_t rr = rho - in.x;
                    const uint32_t rz = __umul24(rr & 255u, in.y) >> 16, ry = rr - __umul24(rz, in.w & 15u);
                    const int dy = (int)((in.w >> 8) & 15u) - 8 + (int)ry, dz = (int)((in.w >> 12) & 15u) - 8 + (int)rz;
                    const uint32_t ady = min((uint32_t)abs(dy), 5u), adz = min((uint32_t)abs(dz), 5u);
                    win[u] = on && !(in.z & (1u << 27));
                    sh[u] = on && (int)ady <= rs && (int)adz <= rs;
                    // the window row: four quads (what falls outside the tile
                    // goes to the halo; the table is the identity past the
                    // window's end)
                    const u64x2 *mrow = reinterpret_cast<const u64x2 *>(mt[(in.z >> 28) & 3u][ady + 6u * adz]);
                    m01[u] = mrow[0];
                    m23[u] = mrow[1];
                    qa[u] = (in.z & 0x7FFu) + __umul24(kTilePq, ry) + __umul24(kTileLayer, rz);
                    // the shadow row: its 7 cells from lx - 3 as bits from
                    // the pair's first cell
                    m7[u] = smask[sh[u] ? ((in.z >> 22) & 31u) * kShadowRows + (uint32_t)(dy + 3) + 7u * (uint32_t)(dz + 3)
                                        : 0u];
                    shf[u] = (in.w >> 4) & 7u;
                    ca[u] = ((in.z >> 11) & 0x7FFu) + __umul24(kCntPitch, ry) + __umul24(kCntLayer, rz);
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    if (win[u]) {
                        unsigned long long *sp = reinterpret_cast<unsigned long long *>(&stamp[qa[u]]);
                        atomicAnd(sp, m01[u].x);
                        atomicAnd(sp + 1, m01[u].y);
                        atomicAnd(sp + 2, m23[u].x);
                        atomicAnd(sp + 3, m23[u].y);
                    }
                    if (sh[u]) {
                        // one count byte a cell, added to two pairs of count
                        // words (a byte cannot carry: at most 255 hits a round)
                        const uint32_t bits = m7[u] << shf[u];
                        unsigned long long *cp = reinterpret_cast<unsigned long long *>(&cnt[ca[u]]);
                        atomicAdd(cp, (unsigned long long)spread4(bits & 15u) |
                                          ((unsigned long long)spread4((bits >> 4) & 15u) << 32));
                        atomicAdd(cp + 1, (unsigned long long)spread4((bits >> 8) & 15u) |
                                              ((unsigned long long)spread4(bits >> 12) << 32));
                    }
                }
            }
            lds_barrier();
            for (uint32_t c = threadIdx.x; c < n_blocks; c += kTileThreads) starts[c] = 0ull;   // for the next round
            // the prefetched values taken into registers now, before the
            // plane loads below are issued
            ent_cur = pe;
            asm volatile("" : "+v"(ent_cur.x), "+v"(ent_cur.y), "+v"(ent_cur.z), "+v"(ent_cur.w));
            // the round's merge (a thread merges the same quads of a tile in
            // every round, so the next round of the same tile loads what this
            // thread stored: program order)
            issue(X0, Y0, Z0, g);
            if (!more) wk_nn = vload(a.work, wi + 2u * G, wi + 2u * G < n_work);
            finish();
        }
        wi += G;
        wk = wk_next;
        wk_next = wk_nn;
    }
}

// ========================================================== mesh export ===
// Marching Cubes of the zero level of the signed distance d = (s ? +1 : -1) *
// popcount(mask) (the mesh export at iso = 0.0 of the paper's pipeline, Sec.
// III). A corner is inside when d < 0, i.e. its sign bit is clear and its mask
// is not empty. Crossed edges take their vertex at t = d_lo / (d_lo - d_hi)
// along the edge, every coordinate one fp32 operation at a time.
// A wavefront takes a run of 64 voxels of one grid row pair (j, j + 1) and
// walks it up through the box in z: each step loads one new layer (two rows,
// both planes: four coalesced loads per lane) and takes the x + 1 corners from
// the next lane, so lanes 0-62 hold cubes and every voxel is read about twice.
// A wavefront walks each 64-step chunk of its run twice: counting, then, with
// the chunk's room reserved by one atomic, writing the triangles of the steps
// that have any; the triangles of a call therefore come out in no fixed order.
constexpr int kMeshThreads = 256;
constexpr uint32_t kMeshRun = 63;     // cubes per wavefront run (lane 63 only lends its corners)

__device__ __forceinline__ uint32_t mesh_low_corner(uint32_t e) {
    const uint32_t a = e >> 2, r = e & 3u;
    return a == 0u ? 2u * r : a == 1u ? ((r & 1u) | ((r & 2u) << 1)) : r;
}

__global__ __launch_bounds__(kMeshThreads) void k_mesh(MeshArgs m) {
    constexpr uint32_t kTabWords = 256 * (kMeshCaseBytes + kMeshTriBytes) / 4;
    static_assert(sizeof(MeshTable) == 4 * kTabWords, "MeshTable layout");
    __shared__ uint32_t tab[kTabWords];
    for (uint32_t i = threadIdx.x; i < kTabWords; i += blockDim.x) tab[i] = m.table[i];
    __syncthreads();
    auto tb = [&](uint32_t cs, uint32_t k) { return (tab[cs * (kMeshCaseBytes / 4) + k / 4] >> (8 * (k % 4))) & 255u; };
    auto tt = [&](uint32_t cs, uint32_t k) {   // the triangle list (kMeshTriBytes per case, after b)
        const uint32_t w = 256u * (kMeshCaseBytes / 4) + cs * (kMeshTriBytes / 4) + k / 4;
        return (tab[w] >> (8 * (k % 4))) & 255u;
    };
    const uint32_t l = lane();
    const uint32_t runs_x = (m.nc[0] + kMeshRun - 1) / kMeshRun;
    const uint64_t n_runs = (uint64_t)runs_x * m.nc[1];
    const uint64_t plane = (uint64_t)m.nx * m.ny;
    const uint32_t wpb = blockDim.x >> 6;
    const uint32_t wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint64_t run = (uint64_t)blockIdx.x * wpb + wid; run < n_runs; run += (uint64_t)gridDim.x * wpb) {
        const uint32_t rx = (uint32_t)(run % runs_x), ry = (uint32_t)(run / runs_x);
        const uint32_t i = m.lo[0] + rx * kMeshRun + l;          // this lane's voxel column
        const uint32_t j = m.lo[1] + ry;
        const bool has_voxel = rx * kMeshRun + l <= m.nc[0];      // voxel i inside the box
        const bool has_cube = l < kMeshRun && rx * kMeshRun + l < m.nc[0];
        // d of the lane's two voxels (rows j, j + 1) in a layer
        auto layer = [&](uint32_t k, int &a, int &b) {
            a = b = 32;
            if (!has_voxel) return;
            const uint64_t v = i + (uint64_t)m.nx * j + plane * k;
            const uint32_t ma = m.mask[v], pa = m.packed[v];
            const uint32_t mb = m.mask[v + m.nx], pb = m.packed[v + m.nx];
            a = (pa >> 31) ? __popc(ma) : -__popc(ma);
            b = (pb >> 31) ? __popc(mb) : -__popc(mb);
        };
        // corners of the cube (i, j, k) from the layers k (pa, pb) and k + 1 (ca, cb)
        auto corners = [&](int pa, int pb, int ca, int cb, int d[8]) {
            d[0] = pa;
            d[1] = __shfl_down(pa, 1, 64);
            d[2] = pb;
            d[3] = __shfl_down(pb, 1, 64);
            d[4] = ca;
            d[5] = __shfl_down(ca, 1, 64);
            d[6] = cb;
            d[7] = __shfl_down(cb, 1, 64);
            uint32_t cs = 0;
#pragma unroll
            for (int c = 0; c < 8; ++c) cs |= (d[c] < 0 ? 1u : 0u) << c;
            return cs;
        };
        // The run goes up in chunks of 64 steps. A first walk counts the
        // chunk's triangles and notes the steps where any lane has some;
        // one atomic reserves the chunk's room (a counter bumped per step
        // would be one hot address); a second walk writes the triangles,
        // visiting only the noted steps. Within the chunk the triangles of
        // a step are contiguous, lane after lane, so the lanes' stores of
        // one step fall on neighbouring lines.
        for (uint32_t k0 = 0; k0 < m.nc[2]; k0 += 64u) {
            const uint32_t kn = min(64u, m.nc[2] - k0);
            uint32_t mine = 0;
            unsigned long long steps = 0;   // wave-uniform: bit s = step k0 + s has triangles
            {
                int pa, pb;
                layer(m.lo[2] + k0, pa, pb);
                for (uint32_t s = 0; s < kn; ++s) {
                    int ca, cb, d[8];
                    layer(m.lo[2] + k0 + s + 1, ca, cb);
                    const uint32_t cs = corners(pa, pb, ca, cb, d);
                    const uint32_t n_t = has_cube ? tb(cs, 0) : 0u;
                    mine += n_t;
                    if (__ballot(n_t != 0u)) steps |= 1ull << s;
                    pa = ca;
                    pb = cb;
                }
            }
            const uint32_t incl = wave_incl_scan_u32(mine);
            const uint32_t total = __shfl(incl, 63, 64);
            if (total == 0u) continue;
            unsigned long long first = 0;
            if (l == 63u) first = atomicAdd(m.count, (unsigned long long)total);
            first = __shfl(first, 63, 64);
            if (!m.out) continue;   // counting only
            unsigned long long run_base = first;   // first slot of the next noted step
            uint32_t loaded = 0xFFFFFFFEu;   // step whose upper layer (pa, pb) holds (none yet)
            int pa = 0, pb = 0;
            const uint32_t i0 = m.lo[0] + rx * kMeshRun;   // voxel column of lane 0
            while (steps) {
                const uint32_t s = (uint32_t)__builtin_ctzll(steps);
                steps &= steps - 1ull;
                const uint32_t k = m.lo[2] + k0 + s;
                if (loaded + 1u != s) layer(k, pa, pb);
                int ca, cb, d[8];
                layer(k + 1, ca, cb);
                const uint32_t cs = corners(pa, pb, ca, cb, d);
                pa = ca;
                pb = cb;
                loaded = s;
                const uint32_t n_t = has_cube ? tb(cs, 0) : 0u;
                const uint32_t inc_t = wave_incl_scan_u32(n_t);
                const uint32_t excl = inc_t - n_t;
                const uint32_t tot = __shfl(inc_t, 63, 64);
                // The step's triangles are written one per lane, so that the
                // whole wavefront works and its stores are contiguous:
                // triangle t belongs to the last cube (lane) c whose first
                // triangle number excl[c] <= t, as its number t - excl[c].
                for (uint32_t t0 = 0; t0 < tot; t0 += 64u) {
                    const uint32_t t = t0 + l;
                    uint32_t c = 0;
#pragma unroll
                    for (uint32_t b = 32u; b; b >>= 1)
                        if ((uint32_t)__shfl((int)excl, (int)(c + b), 64) <= t) c += b;
                    const uint32_t jt = t - (uint32_t)__shfl((int)excl, (int)c, 64);
                    const uint32_t ccs = (uint32_t)__shfl((int)cs, (int)c, 64);
                    int dd[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) dd[q] = __shfl(d[q], (int)c, 64);
                    if (t >= tot) continue;
                    const uint32_t ic = i0 + c;
                    // vertex of crossed edge e of cube (ic, j, k)
                    auto vtx = [&](uint32_t e, float &x, float &y, float &z) {
                        const uint32_t a = e >> 2, clo = mesh_low_corner(e), chi = clo | (1u << a);
                        const uint32_t u[3] = {ic + (clo & 1u), j + ((clo >> 1) & 1u), k + (clo >> 2)};
                        float cc[3];
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            const float h = (float)u[q] + 0.5f;
                            const float hs = h * m.s;
                            cc[q] = m.origin[q] + hs;
                        }
                        const float dlo = (float)dd[clo], dhi = (float)dd[chi];
                        const float den = dlo - dhi;
                        const float tv = dlo / den;
                        const float ts = tv * m.s;
                        cc[a] = cc[a] + ts;
                        x = cc[0];
                        y = cc[1];
                        z = cc[2];
                    };
                    float v[9];
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const uint32_t code = tt(ccs, 3u * jt + (uint32_t)q);
                        if (code & kMeshCentre) {
                            // the centre of the loop whose header is at byte p: the
                            // mean of its vertices, summed in loop order
                            const uint32_t p = code & 127u, mm = tb(ccs, p) & 15u;
                            float sx, sy, sz;
                            vtx(tb(ccs, p + 1u), sx, sy, sz);
                            for (uint32_t w = 1; w < mm; ++w) {
                                float x, y, z;
                                vtx(tb(ccs, p + 1u + w), x, y, z);
                                sx = sx + x;
                                sy = sy + y;
                                sz = sz + z;
                            }
                            const float fm = (float)mm;
                            v[3 * q + 0] = sx / fm;
                            v[3 * q + 1] = sy / fm;
                            v[3 * q + 2] = sz / fm;
                        } else {
                            vtx(code, v[3 * q + 0], v[3 * q + 1], v[3 * q + 2]);
                        }
                    }
                    const unsigned long long slot = run_base + t;
                    if (slot < m.cap) {
                        float *o = m.out + 9ull * slot;
#pragma unroll
                        for (int q = 0; q < 9; ++q) o[q] = v[q];
                    }
                }
                run_base += tot;
            }
        }
    }
}

// Point export: the centres of the occupied contact voxels (a return landed
// there, mask 0, and the hit counter confirmed it, sign 0). A wavefront takes
// kPointRows consecutive rows of the box: a counting pass (kPointPieces
// 64-voxel pieces of a row at a time: all their mask loads, then the counter
// loads where a mask is 0, then one wait and the ballots), one atomic to
// reserve the group's room, then the writing pass with the lanes' ranks from
// the ballots: kept in LDS by the counting pass where the group's rows have
// at most kPointKeep pieces (rows of up to 2048 voxels), else loaded again.
constexpr uint32_t kPointRows = 8;
constexpr int kPointPieces = 16;
constexpr uint32_t kPointKeep = 256;
__global__ __launch_bounds__(kMeshThreads) void k_points(MeshArgs m) {
    const uint32_t l = lane();
    const uint64_t n_rows = (uint64_t)m.nc[1] * m.nc[2];
    const uint64_t n_groups = (n_rows + kPointRows - 1) / kPointRows;
    const uint32_t wpb = blockDim.x >> 6;
    const uint32_t wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned long long below = l ? ((1ull << l) - 1ull) : 0ull;
    const uint32_t W = m.nc[0];
    __shared__ unsigned long long s_bal[kMeshThreads / 64][kPointKeep];   // a wavefront's ballots, in order
    // pieces of a row, in whole steps
    const uint32_t row_pieces = (W + 64u * kPointPieces - 1u) / (64u * kPointPieces) * kPointPieces;
    // ballots of the occupied voxels of row r, pieces x0 .. x0 + 64 kPointPieces - 1
    auto ballots = [&](uint64_t r, uint32_t x0, unsigned long long bal[kPointPieces]) {
        const uint32_t j = m.lo[1] + (uint32_t)(r % m.nc[1]), k = m.lo[2] + (uint32_t)(r / m.nc[1]);
        const uint64_t base = m.lo[0] + (uint64_t)m.nx * (j + (uint64_t)m.ny * k);
        uint32_t mk[kPointPieces], pk[kPointPieces];
#pragma unroll
        for (int u = 0; u < kPointPieces; ++u) {   // (every lane loads: past the row's end, its last voxel)
            const uint32_t x = x0 + 64u * (uint32_t)u + l;
            const uint32_t v = m.mask[base + min(x, W - 1u)];
            mk[u] = x < W ? v : 1u;
        }
#pragma unroll
        for (int u = 0; u < kPointPieces; ++u) {   // the counter only where the mask is 0
            const uint32_t x = x0 + 64u * (uint32_t)u + l;
            pk[u] = 0x80000000u;
            if (mk[u] == 0u) pk[u] = m.packed[base + x];
        }
        // (all the counter loads are issued before the first is used)
#pragma unroll
        for (int u = 0; u < kPointPieces; ++u) asm volatile("" : "+v"(pk[u]));
#pragma unroll
        for (int u = 0; u < kPointPieces; ++u) bal[u] = __ballot(mk[u] == 0u && (pk[u] >> 31) == 0u);
    };
    for (uint64_t grp = (uint64_t)blockIdx.x * wpb + wid; grp < n_groups; grp += (uint64_t)gridDim.x * wpb) {
        const uint64_t r0 = grp * kPointRows, r1 = min(r0 + kPointRows, n_rows);
        const bool keep = (uint64_t)(r1 - r0) * row_pieces <= kPointKeep;
        uint32_t cnt = 0;
        for (uint64_t r = r0; r < r1; ++r)
            for (uint32_t x0 = 0; x0 < W; x0 += 64u * kPointPieces) {
                unsigned long long bal[kPointPieces];
                ballots(r, x0, bal);
                const uint32_t p0 = (uint32_t)(r - r0) * row_pieces + x0 / 64u;
#pragma unroll
                for (int u = 0; u < kPointPieces; ++u) {
                    cnt += (uint32_t)__popcll(bal[u]);
                    if (keep && l == (uint32_t)u) s_bal[wid][p0 + (uint32_t)u] = bal[u];
                }
            }
        if (cnt == 0u) continue;
        unsigned long long first = 0;
        if (l == 0u) first = atomicAdd(m.count, (unsigned long long)cnt);
        first = __shfl(first, 0, 64);
        if (!m.out) continue;   // counting only
        for (uint64_t r = r0; r < r1; ++r) {
            const uint32_t j = m.lo[1] + (uint32_t)(r % m.nc[1]), k = m.lo[2] + (uint32_t)(r / m.nc[1]);
            for (uint32_t x0 = 0; x0 < W; x0 += 64u * kPointPieces) {
                unsigned long long bal[kPointPieces];
                if (keep) {   // (this wavefront's own LDS writes, in program order)
                    const uint32_t p0 = (uint32_t)(r - r0) * row_pieces + x0 / 64u;
#pragma unroll
                    for (int u = 0; u < kPointPieces; ++u) bal[u] = s_bal[wid][p0 + (uint32_t)u];
                } else {
                    ballots(r, x0, bal);
                }
#pragma unroll
                for (int u = 0; u < kPointPieces; ++u) {
                    if ((bal[u] >> l) & 1ull) {
                        const unsigned long long slot = first + (unsigned long long)__popcll(bal[u] & below);
                        if (slot < m.cap) {
                            const uint32_t uu[3] = {m.lo[0] + x0 + 64u * (uint32_t)u + l, j, k};
                            float c[3];
#pragma unroll
                            for (int t = 0; t < 3; ++t) {
                                const float h = (float)uu[t] + 0.5f;
                                const float hs = h * m.s;
                                c[t] = m.origin[t] + hs;
                            }
                            float *o = m.out + 3ull * slot;
                            o[0] = c[0];
                            o[1] = c[1];
                            o[2] = c[2];
                        }
                    }
                    first += (unsigned long long)__popcll(bal[u]);
                }
            }
        }
    }
}

// ================================================================ utility ===
__global__ void k_fill_u32(uint32_t *p, uint32_t v, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_grid_init(uint4 *mask, uint4 *packed, uint64_t n4) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (uint64_t)gridDim.x * blockDim.x) {
        mask[i] = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
        packed[i] = make_uint4(0x80000000u, 0x80000000u, 0x80000000u, 0x80000000u);
    }
}
__global__ void k_read_distance(const uint32_t *mask, const uint32_t *packed, int8_t *out, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const int pc = __popc(mask[i]);
        out[i] = (int8_t)((packed[i] & 0x80000000u) ? pc : -pc);
    }
}

__global__ void k_gather_box(const uint32_t *plane, const uint32_t *packed, uint32_t nx, uint32_t ny, uint32_t lx,
                             uint32_t ly, uint32_t lz, uint32_t sx, uint32_t sy, uint64_t n, void *out) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t x = i % sx, y = (i / sx) % sy, z = i / ((uint64_t)sx * sy);
        const size_t lin = (size_t)(lx + x) + (size_t)nx * ((size_t)(ly + y) + (size_t)ny * (size_t)(lz + z));
        if (packed) {
            const int pc = __popc(plane[lin]);
            ((int8_t *)out)[i] = (int8_t)((packed[lin] & 0x80000000u) ? pc : -pc);
        } else {
            ((uint32_t *)out)[i] = plane[lin];
        }
    }
}

__global__ void k_count_diff(const uint32_t *a, const uint32_t *b, uint64_t n, unsigned long long *count) {
    uint32_t c = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        c += a[i] != b[i];
    c = wave_sum_u32(c);
    if (lane() == 0 && c) atomicAdd(count, (unsigned long long)c);
}

static uint32_t blocks_for(uint64_t n, uint32_t threads, uint32_t cap) {
    uint64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    return (uint32_t)(b > cap ? cap : b);
}

__global__ __launch_bounds__(256) void k_stats_out(PipeArgs a) {
    stats_out(a, reinterpret_cast<const CallInfo *>(a.ctrl + 1));
}
hipError_t launch_stats_out(const PipeArgs &a, hipStream_t st) {
    k_stats_out<<<1, 256, 0, st>>>(a);
    return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t st) {
    if (!n) return hipSuccess;
    k_fill_u32<<<blocks_for(n, 256, 8192), 256, 0, st>>>(p, v, n);
    return hipGetLastError();
}
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, uint64_t n, hipStream_t st) {
    if (!n) return hipSuccess;
    k_fill_u64<<<blocks_for(n, 256, 8192), 256, 0, st>>>(p, v, n);
    return hipGetLastError();
}
hipError_t launch_grid_init(uint32_t *mask, uint32_t *packed, uint64_t n, hipStream_t st) {
    const uint64_t n4 = n / 4;
    if (n4) k_grid_init<<<blocks_for(n4, 256, 16384), 256, 0, st>>>((uint4 *)mask, (uint4 *)packed, n4);
    if (n % 4) {
        k_fill_u32<<<1, 64, 0, st>>>(mask + n4 * 4, 0xFFFFFFFFu, n % 4);
        k_fill_u32<<<1, 64, 0, st>>>(packed + n4 * 4, 0x80000000u, n % 4);
    }
    return hipGetLastError();
}
hipError_t launch_read_distance(const uint32_t *mask, const uint32_t *packed, int8_t *out, uint64_t n, hipStream_t st) {
    if (!n) return hipSuccess;
    k_read_distance<<<blocks_for(n, 256, 16384), 256, 0, st>>>(mask, packed, out, n);
    return hipGetLastError();
}

hipError_t launch_gather_box(const uint32_t *plane, const uint32_t *packed, const uint32_t dims[3],
                             const uint32_t lo[3], const uint32_t hi[3], void *out, hipStream_t st) {
    const uint32_t sx = hi[0] - lo[0], sy = hi[1] - lo[1], sz = hi[2] - lo[2];
    const uint64_t n = (uint64_t)sx * sy * sz;
    if (!n) return hipSuccess;
    k_gather_box<<<blocks_for(n, 256, 16384), 256, 0, st>>>(plane, packed, dims[0], dims[1], lo[0], lo[1], lo[2], sx,
                                                            sy, n, out);
    return hipGetLastError();
}

hipError_t launch_count_diff(const uint32_t *a, const uint32_t *b, uint64_t n, unsigned long long *count,
                             hipStream_t st) {
    if (!n) return hipSuccess;
    k_count_diff<<<blocks_for(n, 256, 8192), 256, 0, st>>>(a, b, n, count);
    return hipGetLastError();
}

// --------------------------------------------------------- apply dispatch ---
#define DBTSDF_BRICKS(X) \
    X(16, 8, 8, 256)     \
    X(32, 8, 8, 256)     \
    X(64, 8, 8, 256)     \
    X(16, 16, 8, 256)    \
    X(32, 16, 8, 256)    \
    X(32, 16, 8, 512)    \
    X(64, 16, 8, 512)    \
    X(32, 16, 16, 512)

typedef void (*apply_fn)(PipeArgs);

// kernel radius 5 (K = 11) and 10 (K = 21, the paper's size) have unrolled
// rows; any other radius takes the generic variant
static apply_fn find_apply(const Tuning &t, int R) {
#define X(BX_, BY_, BZ_, TH_)                                                           \
    if (t.bx == BX_ && t.by == BY_ && t.bz == BZ_ && t.threads == TH_) {                \
        constexpr int mr = max_radius(BX_, BY_, BZ_);                                   \
        if (R == 5 && 5 <= mr) return k_apply_brick<BX_, BY_, BZ_, TH_, 5>;             \
        if (R == 10 && 10 <= mr) return k_apply_brick<BX_, BY_, BZ_, TH_, 10>;          \
        if (R <= mr) return k_apply_brick<BX_, BY_, BZ_, TH_, 0>;                       \
        return nullptr;                                                                 \
    }
    DBTSDF_BRICKS(X)
#undef X
    return nullptr;
}

bool tuning_supported(const Tuning &t, int K) {
    if (t.strategy == DBTSDF_STRATEGY_TILE)   // (the kernel set must have the row kernel's tables too)
        return t.threads == (uint32_t)kTileThreads && t.bx == kTileX && t.by == kTileY && t.bz == kTileZ && K <= 11;
    if (per_point_front(t)) return t.threads >= 64 && t.threads <= 1024 && (t.threads % 64) == 0;
    if (t.strategy != DBTSDF_STRATEGY_BRICK) return false;
    return find_apply(t, (K - 1) / 2) != nullptr;
}

static int apply_blocks_query(const Tuning &t, int K, bool row_kernel, int device);

// The occupancy query costs far more than a launch, so its answer is kept per
// (device, strategy, shape, threads, K, kernel).
int apply_blocks_default(const Tuning &t, int K, bool row_kernel, int device) {
    static std::mutex mu;
    static std::map<std::array<uint32_t, 8>, int> cache;
    const std::array<uint32_t, 8> key = {(uint32_t)device, t.strategy, t.bx, t.by, t.bz, t.threads, (uint32_t)K,
                                         row_kernel ? 1u : 0u};
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    const int v = apply_blocks_query(t, K, row_kernel, device);
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = v;
    return v;
}

static int apply_blocks_query(const Tuning &t, int K, bool row_kernel, int device) {
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) cus = 256;
    // a persistent grid is sized to be fully resident: blocks per CU from the
    // kernel's real register and LDS use (a second round of workgroups would
    // start only when the first has finished its share)
    int per_cu = 0;
    if (t.strategy == DBTSDF_STRATEGY_SORT) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sort_emit_kernel(), kSortThreads, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        return cus * per_cu;
    }
    if (t.strategy == DBTSDF_STRATEGY_ATOMIC) {
        const void *pk = row_kernel ? reinterpret_cast<const void *>(k_apply_points<true>)
                                         : reinterpret_cast<const void *>(k_apply_atomic);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pk, kPtThreads, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        return cus * per_cu;
    }
    if (t.strategy == DBTSDF_STRATEGY_TILE) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(k_apply_tile),
                                                         kTileThreads, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        return cus * per_cu;
    }
    apply_fn f = find_apply(t, (K - 1) / 2);
    if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(f),
                                                           (int)t.threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return cus * per_cu;
}

hipError_t launch_pipeline(const PipeArgs &a, const Tuning &t, uint32_t points_cap, hipStream_t st, int part) {
    const CallInfo *info = reinterpret_cast<const CallInfo *>(a.ctrl + 1);
    const uint32_t pb = blocks_for(points_cap, kPtThreads, 4096);
    const uint32_t sb = blocks_for(points_cap, kSelThreads, 1024);
    uint32_t stat_chunk = 1024;
    while ((uint64_t)stat_chunk * 512 < points_cap) stat_chunk *= 2;
    const bool all = part == kPartAll;
    const bool pre = all || part == kPartPre, apply = all || part == kPartApply, post = all || part == kPartPost;
    if (t.strategy == DBTSDF_STRATEGY_TILE) {
        // front (lists counted), offsets (lists laid out), select and fill,
        // apply; the select pass writes the statistics out
        if (pre) {
            if (a.single_scan) {
                k_front<true, true><<<pb, kPtThreads, 0, st>>>(a, info);
            } else {
                k_upload<<<kCopyBlocks, 256, 0, st>>>(a);
                k_reset<<<8, 256, 0, st>>>(a, info);
                k_front<false, true><<<pb, kPtThreads, 0, st>>>(a, info);
            }
            k_offsets<<<blocks_for(points_cap, kPtThreads, 256), kPtThreads, 0, st>>>(a);
            k_select_fill<<<sb, kSelThreads, 0, st>>>(a, info);
        }
        if (apply) {
            if (!a.tab.row_image) return hipErrorInvalidValue;
            k_apply_tile<<<t.apply_blocks, kTileThreads, 0, st>>>(a);
        }
        (void)post;
        return hipGetLastError();
    }
    if (per_point_front(t)) {
        // three passes: front (one-scan calls copy their descriptors in and
        // clear the counters there), select (writes the statistics out), apply
        // (the sort strategy's apply is sort_apply, which reads counts back)
        if (apply && t.strategy == DBTSDF_STRATEGY_SORT) return hipErrorInvalidValue;
        if (pre) {
            if (a.single_scan) {
                k_front<true, false><<<pb, kPtThreads, 0, st>>>(a, info);
            } else {
                k_upload<<<kCopyBlocks, 256, 0, st>>>(a);
                k_reset<<<8, 256, 0, st>>>(a, info);
                k_front<false, false><<<pb, kPtThreads, 0, st>>>(a, info);
            }
            k_select_atomic<<<sb, kSelThreads, 0, st>>>(a, info);
        }
        // the row kernel covers the kernel sets it has tables for (K <= 11,
        // r_s^2 <= 9, at most 31 bins) and grids with Nx % 4 == 0 whose window
        // offsets fit 32 bits; everything else takes the generic per-row kernel
        if (apply) {
            if (a.row_kernel) {
                if (a.single_scan)
                    k_apply_points<true><<<t.apply_blocks, kPtThreads, 0, st>>>(a, info);
                else
                    k_apply_points<false><<<t.apply_blocks, kPtThreads, 0, st>>>(a, info);
            } else {
                k_apply_atomic<<<t.apply_blocks, kPtThreads, 0, st>>>(a, info);
            }
        }
        (void)post;
        return hipGetLastError();
    }
    apply_fn f = find_apply(t, a.tab.R);
    if (!f) return hipErrorInvalidValue;
    if (pre) {
        k_upload<<<kCopyBlocks, 256, 0, st>>>(a);
        k_reset<<<8, 256, 0, st>>>(a, info);
        k_front<false, false><<<pb, kPtThreads, 0, st>>>(a, info);
        k_select_pairs<<<sb, kSelThreads, 0, st>>>(a, info);
        k_stats<<<blocks_for(points_cap, stat_chunk, 512), kPtThreads, 0, st>>>(a, info, stat_chunk);
        k_offsets<<<blocks_for(points_cap, kPtThreads, 256), kPtThreads, 0, st>>>(a);
        k_fill_pairs<<<pb, kPtThreads, 0, st>>>(a, info);
    }
    if (apply) hipLaunchKernelGGL(f, dim3(t.apply_blocks), dim3(t.threads), 0, st, a);
    if (post) k_download<<<kCopyBlocks, 256, 0, st>>>(a, info);
    return hipGetLastError();
}

hipError_t launch_points(const MeshArgs &m, hipStream_t st) {
    const unsigned long long rows = (unsigned long long)m.nc[1] * m.nc[2];
    if (rows == 0 || m.nc[0] == 0) return hipSuccess;
    const unsigned long long wpb = kMeshThreads / 64, groups = (rows + kPointRows - 1) / kPointRows;
    const uint32_t blocks = (uint32_t)std::min<unsigned long long>((groups + wpb - 1) / wpb, 16384ull);
    k_points<<<blocks, kMeshThreads, 0, st>>>(m);
    return hipGetLastError();
}

hipError_t launch_mesh(const MeshArgs &m, hipStream_t st) {
    if ((unsigned long long)m.nc[0] * m.nc[1] * m.nc[2] == 0) return hipSuccess;
    // one wavefront per run of kMeshRun cubes of a row pair
    const unsigned long long runs = (unsigned long long)((m.nc[0] + kMeshRun - 1) / kMeshRun) * m.nc[1];
    const unsigned long long wpb = kMeshThreads / 64;
    const uint32_t blocks = (uint32_t)std::min<unsigned long long>((runs + wpb - 1) / wpb, 16384ull);
    k_mesh<<<blocks, kMeshThreads, 0, st>>>(m);
    return hipGetLastError();
}

}  // namespace dbtsdf

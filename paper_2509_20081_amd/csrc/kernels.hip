// gfx950 kernels of DB-TSDF scan integration (Sec. III-C of the paper).
//
// One call integrates a set of scans (one for the plain entry point, many for
// the batched one) through this pass sequence on one stream:
//
//   k_reset    zero the per-call counters
//   k_front    per point: fp32 transform into the map frame, validity,
//              voxelisation, K^3 bounds test, direction bin (eq. 2); the
//              first-return-per-voxel rule (Sec. IV-B) by an atomicMin of the
//              point index into a hash table keyed by (scan, voxel)
//   k_select   per point: survivor test; bucketing of survivors by the grid
//              bricks their K^3 cube touches (counting pass, work-item claim)
//   k_offsets  exclusive scan of the per-brick counts -> list offsets
//   k_fill     per survivor: append its index to each touched brick's list;
//              release the hash slots
//   k_apply    persistent: one workgroup owns one brick at a time in LDS,
//              stamps the eq. 3 masks of every listed point with LDS atomicAnd
//              (eq. 4) and counts shadow hits with LDS atomicAdd, then merges
//              the brick into HBM once: mask &= stamp (write skipped when
//              unchanged) and h = min(h + c, H_max) with the eq. 6 sign rule.
//
// Merging per brick is exact because the eq. 4 AND commutes and is
// idempotent, and c unit steps of eq. 5 saturate to min(h + c, H_max) while
// eq. 6 clears the sign iff h_old < T <= h_new; so the grid does not depend on
// the order of points or scans. The alternative "atomic" strategy applies one
// point per wavefront straight into HBM with 32-bit atomics.
//
// Nothing here is a dense contraction, so MFMA is not used; the bound is HBM
// and LDS/atomic throughput.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace dbtsdf {

// ============================================================== helpers ===
__device__ __forceinline__ uint32_t lane() { return __lane_id(); }

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

__device__ __forceinline__ uint32_t front_end(const DevScan &s, const DevGrid &g, const DevTables &t, float px,
                                              float py, float pz, int &vx, int &vy, int &vz, int &bin) {
    if (!__builtin_isfinite(px) || !__builtin_isfinite(py) || !__builtin_isfinite(pz)) return kStInvalid;
    float d[3], w[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float a = s.rot[3 * k + 0] * px;
        const float b = s.rot[3 * k + 1] * py;
        const float c = s.rot[3 * k + 2] * pz;
        const float ab = a + b;
        d[k] = ab + c;
        w[k] = d[k] + s.trans[k];
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

__global__ void k_reset(PipeArgs a, const CallInfo *info) {
    const uint32_t n_sc = info->n_scans * SC_N, n_tc = info->n_grids * TC_N;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_sc + n_tc + 4; i += gridDim.x * blockDim.x) {
        if (i < n_sc) a.scan_ctr[i] = 0ull;
        else if (i < n_sc + n_tc) a.traffic_ctr[i - n_sc] = 0ull;
        else ((uint32_t *)a.ctrl)[i - n_sc - n_tc] = 0u;
    }
}

__global__ __launch_bounds__(kPtThreads) void k_front(PipeArgs a, const CallInfo *info) {
    const uint32_t n = info->n_points, n_scans = info->n_scans;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        const bool live = i < n;
        uint32_t s = 0, st = kStInvalid;
        if (live) {
            s = find_scan(a.scans, n_scans, i);
            const DevScan &sc = a.scans[s];
            const DevGrid &g = a.grids[sc.grid];
            const uint32_t j = i - sc.begin;
            const float px = sc.pts[3 * (size_t)j + 0];
            const float py = sc.pts[3 * (size_t)j + 1];
            const float pz = sc.pts[3 * (size_t)j + 2];
            int vx = 0, vy = 0, vz = 0, bin = 0;
            st = front_end(sc, g, a.tab, px, py, pz, vx, vy, vz, bin);
            uint32_t slot = kNoSlot;
            if (st == kStOk && sc.dedup) {
                const unsigned long long lin =
                    (unsigned long long)vx + (unsigned long long)g.nx * ((unsigned long long)vy + (unsigned long long)g.ny * (unsigned long long)vz);
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
            a.rec[i] = make_uint4((uint32_t)vx, (uint32_t)vy, (uint32_t)vz, (st << 16) | (uint32_t)bin);
            a.pslot[i] = slot;
        }
        wave_add(a.scan_ctr, s, SC_INVALID, live && st == kStInvalid ? 1u : 0u);
        wave_add(a.scan_ctr, s, SC_OOB, live && st == kStOob ? 1u : 0u);
    }
}

// brick span of the cube [c - R, c + R] along one axis with brick side 1 << sh
__device__ __forceinline__ void span(uint32_t c, int R, uint32_t sh, uint32_t &b0, uint32_t &nb) {
    b0 = (c - (uint32_t)R) >> sh;
    nb = ((c + (uint32_t)R) >> sh) - b0 + 1u;
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
    if ((o.r.w >> 16) != kStOk) return o;
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

__global__ __launch_bounds__(kPtThreads) void k_select_brick(PipeArgs a, const CallInfo *info) {
    const uint32_t n = info->n_points;
    const uint32_t shx = __builtin_ctz(a.brick[0]), shy = __builtin_ctz(a.brick[1]), shz = __builtin_ctz(a.brick[2]);
    const int R = a.tab.R;
    // uniform bound on bricks per cube, same for every lane
    const uint32_t mx = 1u + (2u * R + a.brick[0] - 1u) / a.brick[0];
    const uint32_t my = 1u + (2u * R + a.brick[1] - 1u) / a.brick[1];
    const uint32_t mz = 1u + (2u * R + a.brick[2] - 1u) / a.brick[2];
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        const SelectOut o = select_point(a, info, i, i < n);
        uint32_t gi = 0, bx0 = 0, by0 = 0, bz0 = 0, nbx = 0, nby = 0, nbz = 0;
        DevGrid g{};
        if (o.surv) {
            a.rec[i].w = o.r.w | kRecSurvivor;
            gi = a.scans[o.s].grid;
            g = a.grids[gi];
            span(o.r.x, R, shx, bx0, nbx);
            span(o.r.y, R, shy, by0, nby);
            span(o.r.z, R, shz, bz0, nbz);
        }
        for (uint32_t jz = 0; jz < mz; ++jz)
            for (uint32_t jy = 0; jy < my; ++jy)
                for (uint32_t jx = 0; jx < mx; ++jx) {
                    const bool valid = o.surv && jx < nbx && jy < nby && jz < nbz;
                    uint32_t id = 0;
                    bool first = false;
                    if (valid) {
                        id = (bx0 + jx) + g.nbx * ((by0 + jy) + g.nby * (bz0 + jz));
                        first = atomicAdd(&g.brick_cnt[id], 1u) == 0u;
                    }
                    const uint32_t slot = wave_claim(&a.ctrl->n_active, first);
                    if (first) {
                        a.items[slot] = ((unsigned long long)gi << 32) | id;
                        g.brick_slot[id] = slot;
                    }
                }
        wave_add(a.scan_ctr, o.s, SC_DUP, o.dup ? 1u : 0u);
        wave_add(a.scan_ctr, o.s, SC_INT, o.surv ? 1u : 0u);
        wave_add(a.scan_ctr, o.s, SC_SHADOW, o.shadow_n);
    }
}

__global__ __launch_bounds__(kPtThreads) void k_offsets(PipeArgs a) {
    const uint32_t n = a.ctrl->n_active;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t t = base + threadIdx.x;
        uint32_t cnt = 0;
        if (t < n) {
            const unsigned long long it = a.items[t];
            cnt = a.grids[it >> 32].brick_cnt[(uint32_t)it];
        }
        const uint32_t incl = wave_incl_scan_u32(cnt);
        uint32_t wbase = 0;
        if (lane() == 63u) wbase = atomicAdd(&a.ctrl->total_entries, incl);
        wbase = __shfl(wbase, 63, 64);
        if (t < n) {
            a.item_off[t] = wbase + incl - cnt;
            a.item_cur[t] = 0u;
        }
    }
}

__global__ __launch_bounds__(kPtThreads) void k_fill(PipeArgs a, const CallInfo *info) {
    const uint32_t n = info->n_points;
    const uint32_t shx = __builtin_ctz(a.brick[0]), shy = __builtin_ctz(a.brick[1]), shz = __builtin_ctz(a.brick[2]);
    const int R = a.tab.R;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint4 r = a.rec[i];
        const uint32_t slot = a.pslot[i];
        if (slot != kNoSlot) {  // release the dedup slot (every reader is done)
            a.hkeys[slot] = kHashEmpty;
            a.hvals[slot] = 0xFFFFFFFFu;
        }
        if (!(r.w & kRecSurvivor)) continue;
        const uint32_t s = find_scan(a.scans, info->n_scans, i);
        const DevGrid g = a.grids[a.scans[s].grid];
        uint32_t bx0, by0, bz0, nbx, nby, nbz;
        span(r.x, R, shx, bx0, nbx);
        span(r.y, R, shy, by0, nby);
        span(r.z, R, shz, bz0, nbz);
        for (uint32_t jz = 0; jz < nbz; ++jz)
            for (uint32_t jy = 0; jy < nby; ++jy)
                for (uint32_t jx = 0; jx < nbx; ++jx) {
                    const uint32_t id = (bx0 + jx) + g.nbx * ((by0 + jy) + g.nby * (bz0 + jz));
                    const uint32_t it = g.brick_slot[id];
                    const uint32_t pos = a.item_off[it] + atomicAdd(&a.item_cur[it], 1u);
                    a.entries[pos] = i;
                }
    }
}

// --------------------------------------------------------------- apply ---
// One workgroup owns brick (BX, BY, BZ) of one grid at a time. LDS holds the
// brick's AND-accumulated eq. 3 stamp and its shadow hit counts.
template <int BX, int BY, int BZ, int THREADS>
__global__ __launch_bounds__(THREADS) void k_apply_brick(PipeArgs a) {
    constexpr int V = BX * BY * BZ;
    constexpr int WAVES = THREADS / 64;
    __shared__ uint32_t lmask[V];
    __shared__ uint32_t lcnt[V];
    __shared__ uint32_t lut[3 * kMaxK * kMaxK / 4 + 8];   // mask by metric value (n_q <= 3 R^2 + 1)
    __shared__ unsigned long long red[3 * WAVES];

    const DevTables &t = a.tab;
    for (uint32_t q = threadIdx.x; q < t.n_q; q += THREADS) lut[q] = t.mask_by_q[q];
    const int R = t.R;
    const bool l1 = t.metric == DBTSDF_DIST_L1;
    const uint32_t n_items = a.ctrl->n_active;
    const uint32_t w = threadIdx.x >> 6, l = lane();

    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const unsigned long long it = a.items[item];
        const DevGrid g = a.grids[it >> 32];
        const uint32_t brick = (uint32_t)it;
        const uint32_t bxi = brick % g.nbx, byi = (brick / g.nbx) % g.nby, bzi = brick / (g.nbx * g.nby);
        const int x0 = (int)bxi * BX, y0 = (int)byi * BY, z0 = (int)bzi * BZ;
        const uint32_t start = a.item_off[item];
        const uint32_t cnt = g.brick_cnt[brick];

        for (int v = threadIdx.x; v < V; v += THREADS) {
            lmask[v] = 0xFFFFFFFFu;
            lcnt[v] = 0u;
        }
        __syncthreads();

        // stamp: one wavefront per listed point
        for (uint32_t e = w; e < cnt; e += WAVES) {
            const uint32_t pidx = a.entries[start + e];
            const uint4 r = a.rec[pidx];
            const int lx = (int)r.x - x0, ly = (int)r.y - y0, lz = (int)r.z - z0;
            const int xa = max(lx - R, 0), xb = min(lx + R, BX - 1);
            const int ya = max(ly - R, 0), yb = min(ly + R, BY - 1);
            const int za = max(lz - R, 0), zb = min(lz + R, BZ - 1);
            const uint32_t wx = (uint32_t)(xb - xa + 1), wy = (uint32_t)(yb - ya + 1), wz = (uint32_t)(zb - za + 1);
            const uint32_t rpi = 64u / wx;           // rows per wave step
            const uint32_t xi = l % wx, ri = l / wx;
            const bool lane_on = ri < rpi;
            const uint32_t rows = wy * wz;
            const uint32_t mag = ((1u << 20) + wy - 1u) / wy;  // exact r / wy for r < 2^20 / wy
            const int ox = xa + (int)xi - lx;
            const int xx = xa + (int)xi;
            for (uint32_t r0 = 0; r0 < rows; r0 += rpi) {
                const uint32_t rr = r0 + ri;
                if (lane_on && rr < rows) {
                    const uint32_t rz = (rr * mag) >> 20;
                    const uint32_t ry = rr - rz * wy;
                    const int yy = ya + (int)ry, zz = za + (int)rz;
                    const int oy = yy - ly, oz = zz - lz;
                    const uint32_t q = l1 ? (uint32_t)(abs(ox) + abs(oy) + abs(oz)) : (uint32_t)(ox * ox + oy * oy + oz * oz);
                    atomicAnd(&lmask[xx + BX * (yy + BY * zz)], lut[q]);
                }
            }
            const uint32_t bin = r.w & 0xFFFFu;
            const uint32_t s0 = t.sh_start[bin], s1 = t.sh_start[bin + 1];
            for (uint32_t j = s0 + l; j < s1; j += 64u) {
                const uint32_t off = t.sh_off[j];
                const int sx = lx + (int)(off & 255u) - R;
                const int sy = ly + (int)((off >> 8) & 255u) - R;
                const int sz = lz + (int)((off >> 16) & 255u) - R;
                if (sx >= 0 && sx < BX && sy >= 0 && sy < BY && sz >= 0 && sz < BZ)
                    atomicAdd(&lcnt[sx + BX * (sy + BY * sz)], 1u);
            }
        }
        __syncthreads();

        // merge the brick into HBM
        uint32_t um = 0, cm = 0, us = 0;
        for (int v = threadIdx.x; v < V; v += THREADS) {
            const uint32_t m = lmask[v], c = lcnt[v];
            if (m == 0xFFFFFFFFu && c == 0u) continue;
            const uint32_t gx = (uint32_t)(x0 + (v % BX)), gy = (uint32_t)(y0 + (v / BX) % BY), gz = (uint32_t)(z0 + v / (BX * BY));
            if (gx >= g.nx || gy >= g.ny || gz >= g.nz) continue;
            const size_t lin = (size_t)gx + (size_t)g.nx * ((size_t)gy + (size_t)g.ny * gz);
            if (m != 0xFFFFFFFFu) {
                const uint32_t old = g.mask[lin];
                const uint32_t nw = old & m;
                if (nw != old) {
                    g.mask[lin] = nw;
                    ++cm;
                }
                ++um;
            }
            if (c) {
                const uint32_t old = g.packed[lin];
                const uint32_t h0 = old & 0xFFFFu;
                const uint32_t h1 = min(h0 + c, g.hmax);
                uint32_t sign = old & 0x80000000u;
                if (h0 < g.T && h1 >= g.T) sign = 0u;
                const uint32_t nw = sign | h1;
                if (nw != old) g.packed[lin] = nw;
                ++us;
            }
        }
        if (a.count_traffic) {
            const uint32_t su = wave_sum_u32(um), sc = wave_sum_u32(cm), ss = wave_sum_u32(us);
            if (l == 0) {
                red[3 * w + 0] = su;
                red[3 * w + 1] = sc;
                red[3 * w + 2] = ss;
            }
            __syncthreads();
            if (threadIdx.x < 3) {
                unsigned long long tot = 0;
                for (int k = 0; k < WAVES; ++k) tot += red[3 * k + threadIdx.x];
                if (tot) atomicAdd(&a.traffic_ctr[(size_t)g.traffic_slot * TC_N + threadIdx.x], tot);
            }
        }
        if (threadIdx.x == 0) g.brick_cnt[brick] = 0u;  // ready for the next call
        __syncthreads();
    }
}

// ------------------------------------------------------ atomic strategy ---
__global__ __launch_bounds__(kPtThreads) void k_select_atomic(PipeArgs a, const CallInfo *info) {
    const uint32_t n = info->n_points;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        const SelectOut o = select_point(a, info, i, i < n);
        const uint32_t slot = wave_claim(&a.ctrl->n_survivors, o.surv);
        if (o.surv) a.survivors[slot] = i;
        wave_add(a.scan_ctr, o.s, SC_DUP, o.dup ? 1u : 0u);
        wave_add(a.scan_ctr, o.s, SC_INT, o.surv ? 1u : 0u);
        wave_add(a.scan_ctr, o.s, SC_SHADOW, o.shadow_n);
    }
}

// One wavefront per surviving point, straight into HBM: read-first atomicAnd
// (eq. 4) and the guard-bit counter (eqs. 5-6): every add that sees a raw
// count >= H_max is cancelled, and the add that sees T - 1 clears the sign.
// Bits 16-30 absorb the transient overshoot of concurrent adds.
__global__ __launch_bounds__(kPtThreads) void k_apply_atomic(PipeArgs a, const CallInfo *info) {
    const DevTables &t = a.tab;
    const int K = t.K, R = t.R;
    const bool l1 = t.metric == DBTSDF_DIST_L1;
    const uint32_t n_surv = a.ctrl->n_survivors;
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    const uint32_t l = lane();
    const uint32_t wx = (uint32_t)K, rpi = 64u / wx, xi = l % wx, ri = l / wx;
    const bool lane_on = ri < rpi;
    const uint32_t rows = (uint32_t)(K * K);
    const uint32_t mag = ((1u << 20) + wx - 1u) / wx;
    for (uint32_t e = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); e < n_surv; e += waves) {
        const uint32_t i = a.survivors[e];
        const uint4 r = a.rec[i];
        const uint32_t s = find_scan(a.scans, info->n_scans, i);
        const DevGrid g = a.grids[a.scans[s].grid];
        const int ox = (int)xi - R;
        for (uint32_t r0 = 0; r0 < rows; r0 += rpi) {
            const uint32_t rr = r0 + ri;
            if (lane_on && rr < rows) {
                const uint32_t rz = (rr * mag) >> 20;
                const uint32_t ry = rr - rz * wx;
                const int oy = (int)ry - R, oz = (int)rz - R;
                const uint32_t q = l1 ? (uint32_t)(abs(ox) + abs(oy) + abs(oz)) : (uint32_t)(ox * ox + oy * oy + oz * oz);
                const uint32_t m = t.mask_by_q[q];
                const size_t lin = (size_t)(r.x + ox) + (size_t)g.nx * ((size_t)(r.y + oy) + (size_t)g.ny * (size_t)(r.z + oz));
                const uint32_t old = g.mask[lin];
                if ((old & m) != old) atomicAnd(&g.mask[lin], m);
            }
        }
        const uint32_t bin = r.w & 0xFFFFu;
        for (uint32_t j = t.sh_start[bin] + l; j < t.sh_start[bin + 1]; j += 64u) {
            const uint32_t off = t.sh_off[j];
            const int sx = (int)r.x + (int)(off & 255u) - R;
            const int sy = (int)r.y + (int)((off >> 8) & 255u) - R;
            const int sz = (int)r.z + (int)((off >> 16) & 255u) - R;
            const size_t lin = (size_t)sx + (size_t)g.nx * ((size_t)sy + (size_t)g.ny * (size_t)sz);
            const uint32_t old = atomicAdd(&g.packed[lin], 1u);
            const uint32_t raw = old & 0x7FFFFFFFu;
            if (raw >= g.hmax) atomicSub(&g.packed[lin], 1u);
            else if (g.T >= 1u && raw == g.T - 1u) atomicAnd(&g.packed[lin], 0x7FFFFFFFu);
        }
    }
}

__global__ __launch_bounds__(kPtThreads) void k_clear_hash(PipeArgs a, const CallInfo *info) {
    const uint32_t n = info->n_points;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t slot = a.pslot[i];
        if (slot != kNoSlot) {
            a.hkeys[slot] = kHashEmpty;
            a.hvals[slot] = 0xFFFFFFFFu;
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
#define DBTSDF_BRICKS(X)     \
    X(32, 16, 8, 256)        \
    X(32, 16, 8, 512)        \
    X(32, 16, 16, 256)       \
    X(32, 16, 16, 512)       \
    X(32, 32, 16, 512)       \
    X(64, 16, 8, 256)        \
    X(64, 16, 8, 512)        \
    X(32, 8, 8, 256)         \
    X(16, 16, 16, 256)       \
    X(16, 16, 8, 256)

typedef void (*apply_fn)(PipeArgs);

static apply_fn find_apply(const Tuning &t) {
#define X(BX_, BY_, BZ_, TH_) \
    if (t.bx == BX_ && t.by == BY_ && t.bz == BZ_ && t.threads == TH_) return k_apply_brick<BX_, BY_, BZ_, TH_>;
    DBTSDF_BRICKS(X)
#undef X
    return nullptr;
}

bool tuning_supported(const Tuning &t, int K) {
    if (t.strategy == DBTSDF_STRATEGY_ATOMIC) return t.threads >= 64 && t.threads <= 1024 && (t.threads % 64) == 0;
    if (t.strategy != DBTSDF_STRATEGY_BRICK) return false;
    (void)K;
    return find_apply(t) != nullptr;
}

int apply_blocks_default(const Tuning &t, int device) {
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) cus = 256;
    if (t.strategy == DBTSDF_STRATEGY_ATOMIC) return cus * 8;
    const size_t lds = (size_t)t.bx * t.by * t.bz * 8 + 4 * 1024;
    int per_cu = (int)((160 * 1024) / lds);
    const int by_threads = 2048 / (int)t.threads;
    if (per_cu > by_threads) per_cu = by_threads;
    if (per_cu < 1) per_cu = 1;
    return cus * per_cu;
}

hipError_t launch_pipeline(const PipeArgs &a, const Tuning &t, uint32_t points_cap, hipStream_t st,
                           hipEvent_t ev_apply0, hipEvent_t ev_apply1) {
    const CallInfo *info = reinterpret_cast<const CallInfo *>(a.ctrl + 1);
    const uint32_t pb = blocks_for(points_cap, kPtThreads, 4096);
    k_reset<<<8, 256, 0, st>>>(a, info);
    k_front<<<pb, kPtThreads, 0, st>>>(a, info);
    if (t.strategy == DBTSDF_STRATEGY_ATOMIC) {
        k_select_atomic<<<pb, kPtThreads, 0, st>>>(a, info);
        if (ev_apply0) (void)hipEventRecord(ev_apply0, st);
        k_apply_atomic<<<t.apply_blocks, kPtThreads, 0, st>>>(a, info);
        if (ev_apply1) (void)hipEventRecord(ev_apply1, st);
        k_clear_hash<<<pb, kPtThreads, 0, st>>>(a, info);
        return hipGetLastError();
    }
    apply_fn f = find_apply(t);
    if (!f) return hipErrorInvalidValue;
    k_select_brick<<<pb, kPtThreads, 0, st>>>(a, info);
    k_offsets<<<blocks_for(a.items_cap, kPtThreads, 1024), kPtThreads, 0, st>>>(a);
    k_fill<<<pb, kPtThreads, 0, st>>>(a, info);
    if (ev_apply0) (void)hipEventRecord(ev_apply0, st);
    hipLaunchKernelGGL(f, dim3(t.apply_blocks), dim3(t.threads), 0, st, a);
    if (ev_apply1) (void)hipEventRecord(ev_apply1, st);
    return hipGetLastError();
}

}  // namespace dbtsdf
